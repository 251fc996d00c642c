// Host runtime of the C ABI declared in include/fcs.h: context, validated
// uploads of the flattened geometry and parametrization, workspace, the
// launch sequence of one batch (optionally captured in a hipGraph), the
// per-event launch loop, and the adjoint.
//
// One translation unit holds the whole library (no relocatable device code).
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fcs.h"
#include "fcs_kernels.hpp"

namespace {
// A roctx range around an entry point's work: rocprofv3 --marker-trace shows
// each call of the library beside its kernels.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};
}  // namespace

using fcsk::Counters;
using fcsk::Params;

namespace {

std::string g_create_error = "no error";

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct GraphKey {
    long long n_particles, n_events;
    int mode, grid, part, f64, win;
    bool operator<(const GraphKey& o) const
    {
        return std::tie(n_particles, n_events, mode, grid, part, f64, win) <
               std::tie(o.n_particles, o.n_events, o.mode, o.grid, o.part, o.f64, o.win);
    }
};

// device block: Params, then Counters at kCtrOffset
constexpr size_t kCtrOffset = (sizeof(Params) + 255) & ~(size_t)255;
constexpr size_t kBlockBytes = kCtrOffset + ((sizeof(Counters) + 255) & ~(size_t)255);

}  // namespace

constexpr int kRing = 256;     // pinned parameter blocks: how many calls the host may run ahead
constexpr int kMaxWindows = 256;  // cell windows of the window pass per geometry (staged in LDS)
// the window pass is used for launches of at least this many particles per
// event on average (hard-scatter and pile-up events; single-particle events
// keep the packed tiles)
constexpr long long kWinMinParticlesPerEvent = 64;
constexpr int kProfRing = 64;     // event pairs of profiled asynchronous calls
constexpr int kHostCopyWgs = 2;   // workgroups of the copy kernel to host buffers (~50 GB/s)

struct fcs_ctx {
    int device = 0;
    bool dry = false;  // FCS_DEVICE_NONE: argument checks only
    int n_cu = 0;
    char name[64] = {0};
    hipStream_t stream = nullptr;
    std::vector<int32_t> h_task_n;  // per-task launch form: an event's hit counts
    hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_in = nullptr;
    hipEvent_t ev_k0 = nullptr, ev_k1 = nullptr;  // around the hit kernel
    hipEvent_t ev_p0 = nullptr, ev_p1 = nullptr;  // around a profiled launch sequence
    std::string err = "no error";
    long long held = 0;

    // geometry
    bool has_geom = false;
    long long n_cells = 0;
    int n_layers = 0, n_regions = 0;
    DevBuf g_eta_lo, g_eta_hi, g_inv_deta, g_inv_dphi, g_phi_lo, g_neta, g_nphi, g_offset,
        g_inv_r, g_cell_id;
    DevBuf g_layers, g_regions;  // lookup records staged in LDS by the hit kernels
    DevBuf g_windows;            // cell windows of the window pass (fcsk::WinRec)
    int n_windows = 0;

    // parametrization (the tables calls use)
    bool has_param = false;
    int n_types = 0, n_ebins = 0, n_etabins = 0;
    float r_max = 0.f;
    long long n_hist = 0;
    DevBuf p_e_edges, p_eta_edges, p_alpha, p_weights, p_cum, p_guide;
    // a second table set filled by fcs_load_parametrization_async on the copy
    // stream; the next call switches to it (its stream waits for ev_loaded)
    bool pending = false;
    int s_types = 0, s_ebins = 0, s_etabins = 0;
    float s_rmax = 0.f;
    long long s_hist = 0;
    DevBuf s_e_edges, s_eta_edges, s_alpha, s_weights, s_cum, s_guide;
    char* h_tab = nullptr;  // pinned host staging of the tables being loaded
    size_t h_tab_bytes = 0;
    // ev_spare_free: recorded when a set becomes the spare, after every call
    // that may read it
    hipEvent_t ev_loaded = nullptr, ev_spare_free = nullptr;
    bool load_in_flight = false;

    // workspace
    DevBuf w_particles, w_evoff, w_override, w_task_n, w_task_ehit, w_part_ev, w_part_p,
        w_part_set, w_blk_sums, w_blk_offs, w_grp, w_task_hoff, w_chunks, w_small_rec,
        w_tile_first, w_cells, w_flags, w_seg_off, w_seg_blk, w_blk_list, w_queue, w_params,
        w_acc_el, w_acc_bins, w_hist_mark;
    long long cells_events = 0;  // events the accumulator holds (kept zero)
    long long flag_events = 0;
    long long chunk_cap = 0;
    // staging of host outputs
    DevBuf o_cells, o_ids, o_e, o_evoff, o_heta, o_hphi, o_he, o_hcell, o_thoff, o_counts,
        o_elayer;

    // ring of pinned host blocks, each holding the Params of a launch
    // followed by its Counters; one copy uploads both (the counters zeroed),
    // and a synchronous launch reads its counters back into the same block.
    // A block is reused only after the copy that read it has completed, so
    // asynchronous calls never overwrite parameters still to be uploaded.
    char* h_ring = nullptr;
    hipEvent_t ring_ev[kRing] = {};
    bool ring_used[kRing] = {};
    int ring_next = 0;
    // asynchronous calls: running totals on the device, hit-kernel timing
    // events of profiled calls not yet read
    DevBuf w_async;
    hipEvent_t ev_done = nullptr;
    hipEvent_t prof_ev[kProfRing][2] = {};
    int prof_head = 0, prof_count = 0;
    double async_kernel_ms = 0.0;
    std::map<GraphKey, hipGraphExec_t> graphs;
    // asynchronous calls with pinned host outputs: the batch compacts into
    // one of two device staging sets (used in turn) and a copy kernel on
    // copy_stream writes the lists to the host while the next batch runs
    hipStream_t copy_stream = nullptr;
    // the window pass runs on win_stream beside the task scans (it needs
    // only the setup pass's outputs); forked after the setup pass and
    // joined before the compaction, also inside captured graphs
    hipStream_t win_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    DevBuf hs_ids[2], hs_e[2], hs_off[2];
    hipEvent_t ev_staged[2] = {}, ev_copied[2] = {};
    bool copy_pending[2] = {};
    int hs_next = 0;
    // the copy of the last such call, not yet enqueued: it waits for the
    // next call's setup pass (ev_pre), so that it runs beside that call's
    // hit kernels; every other entry point enqueues it first
    struct HostCopy {
        int hs, wgs;
        int64_t *h_ids, *h_off;
        float* h_e;
        long long n_events, m;
    } dc{};
    bool copy_deferred = false;
    hipEvent_t ev_pre = nullptr;
    // the copy of an earlier batch out of the staging set this call reuses:
    // the call's stream waits for it just before the compaction writes the
    // set (its setup pass and hit kernels run beside the copy)
    hipEvent_t post_wait = nullptr;
    // the work queue in the workspace: the device inputs and options it was
    // built from and its parameter block; an adjoint call with
    // reuse_forward_queue and the same inputs skips the setup and the scans.
    // Any call that rebuilds or may overwrite the workspace clears q_valid.
    struct QueueKey {
        const void *particles, *evoff, *override_;
        long long n_events, n_particles, ev_base;
        unsigned long long seed;
        float scale;
        int cap;
        double min_e;
        int chunk, big, tile;
        bool operator==(const QueueKey& o) const
        {
            return std::tie(particles, evoff, override_, n_events, n_particles, ev_base, seed, scale, cap,
                            min_e, chunk, big, tile) ==
                   std::tie(o.particles, o.evoff, o.override_, o.n_events, o.n_particles, o.ev_base, o.seed,
                            o.scale, o.cap, o.min_e, o.chunk, o.big, o.tile);
        }
    };
    bool q_valid = false;
    QueueKey q_key{};
    Params q_params{};
    // device address of the Params block (Counters at kCtrOffset) that the
    // kernels of the current call read: w_params, or the start of the
    // no-allocation scratch array
    char* cur_params = nullptr;
    // this device's scratch array for fcs_simulate_events_noalloc (its
    // address looked up once per device at the first fcs_create there)
    char* scratch = nullptr;
};

namespace {

int fail(fcs_ctx* c, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_create_error = buf;
    return code;
}

#define HIPCHK(ctx, call)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, FCS_E_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                 \
    } while (0)

void release(fcs_ctx* c, DevBuf& b)
{
    if (b.p) {
        (void)hipFree(b.p);
        c->held -= (long long)b.bytes;
    }
    b.p = nullptr;
    b.bytes = 0;
}

// The next pinned parameter block of the ring (waits until the copy that
// last read it has completed); ring_sent() after its upload is enqueued.
char* ring_take(fcs_ctx* c)
{
    const int i = c->ring_next;
    if (c->ring_used[i] && hipEventSynchronize(c->ring_ev[i]) != hipSuccess) return nullptr;
    return c->h_ring + (size_t)i * kBlockBytes;
}

int ring_sent(fcs_ctx* c)
{
    const int i = c->ring_next;
    HIPCHK(c, hipEventRecord(c->ring_ev[i], c->stream));
    c->ring_used[i] = true;
    c->ring_next = (i + 1) % kRing;
    return FCS_OK;
}

// grow-only device buffer; contents are not preserved
int ensure(fcs_ctx* c, DevBuf& b, size_t bytes, bool* grown = nullptr)
{
    if (grown) *grown = false;
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return FCS_OK;
    // the old buffer may still be read by enqueued (asynchronous) work
    if (b.p && c->stream) (void)hipStreamSynchronize(c->stream);
    release(c, b);
    size_t want = bytes + bytes / 8;
    want = (want + 255) & ~(size_t)255;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(c, FCS_E_NOMEM, "device allocation of %zu bytes failed", want);
    }
    b.bytes = want;
    c->held += (long long)want;
    if (grown) *grown = true;
    return FCS_OK;
}

template <typename T>
int upload(fcs_ctx* c, DevBuf& b, const T* src, size_t n)
{
    int rc = ensure(c, b, n * sizeof(T));
    if (rc) return rc;
    if (n) HIPCHK(c, hipMemcpy(b.p, src, n * sizeof(T), hipMemcpyHostToDevice));
    return FCS_OK;
}

unsigned grid_for(long long n, int block) { return (unsigned)((n + block - 1) / block); }

void drop_graphs(fcs_ctx* c)
{
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

bool finite_pos(float v) { return std::isfinite(v) && v > 0.f; }

// Enqueue the copy of an asynchronous call's compacted lists (staging set
// dc.hs) to its pinned host buffers on the copy stream, after `after`.
int enqueue_host_copy(fcs_ctx* c, const fcs_ctx::HostCopy& dc, hipEvent_t after)
{
    const int hs = dc.hs;
    HIPCHK(c, hipStreamWaitEvent(c->copy_stream, after, 0));
    const int64_t* d_ids = (const int64_t*)c->hs_ids[hs].p;
    const float* d_e = (const float*)c->hs_e[hs].p;
    const int64_t* d_off = (const int64_t*)c->hs_off[hs].p;
    if (dc.wgs > 0) {
        // a copy kernel of a few workgroups stores what the batch wrote
        // through the buffers' device mapping
        hipLaunchKernelGGL(fcsk::k_copy_out, dim3(dc.wgs), dim3(fcsk::kBlock), 0, c->copy_stream, d_ids, d_e,
                           d_off, dc.h_ids, dc.h_e, dc.h_off, dc.n_events, dc.m);
        HIPCHK(c, hipGetLastError());
    } else {
        // the runtime's copies of the offsets and of m entries of each list
        HIPCHK(c, hipMemcpyAsync(dc.h_off, d_off, (size_t)(dc.n_events + 1) * 8, hipMemcpyDeviceToHost,
                                 c->copy_stream));
        if (dc.m) {
            HIPCHK(c, hipMemcpyAsync(dc.h_ids, d_ids, (size_t)dc.m * 8, hipMemcpyDeviceToHost, c->copy_stream));
            HIPCHK(c, hipMemcpyAsync(dc.h_e, d_e, (size_t)dc.m * 4, hipMemcpyDeviceToHost, c->copy_stream));
        }
    }
    HIPCHK(c, hipEventRecord(c->ev_copied[hs], c->copy_stream));
    c->copy_pending[hs] = true;
    return FCS_OK;
}

// Enqueue a deferred copy: after `after` (recorded on the context's stream
// after the next batch's setup pass), else after the batch that staged it.
int flush_host_copy(fcs_ctx* c, hipEvent_t after = nullptr)
{
    if (!c->copy_deferred) return FCS_OK;
    c->copy_deferred = false;
    return enqueue_host_copy(c, c->dc, after ? after : c->ev_staged[c->dc.hs]);
}

// pinned host memory that the device can write through its mapping
bool pinned_host(const void* p)
{
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeHost && a.devicePointer != nullptr;
}

// ------------------------------------------ no-allocation scratch array ---
// fcs_simulate_events_noalloc keeps every device buffer of a call other than
// its inputs, outputs and the loaded tables (parameter block, counters,
// work-queue tickets, task arrays, work queue, block counts, compaction
// lists, private accumulator) in this array.  Each GPU the library runs on
// holds its own copy until the process ends.  In host code the name is not a
// device address: its address on a device is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept in g_scratch_dev.
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_dev[kMaxDevices] = {};

// the scratch array's address on `device` (current); nullptr on failure
char* scratch_on_device(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_dev[device] = (char*)ptr;
    }
    return g_scratch_dev[device];
}

// The smallest hit energy E_layer / n a call may produce: FLT_MIN, and with
// the energy fluctuation FLT_MIN 2^26 (its factor exceeds 2^-26), so that every
// deposited energy is a normal FP32 number.  The deposits count a cell as new
// when an atomic add finds it at zero, which a flushed subnormal addend would
// break.  A call's own layer energies are at least min_layer_energy_mev,
// checked against nhit_cap times this bound; an override is checked per
// (particle, layer) with hits on the device.
double min_hit_energy(const fcs_sim_options* o)
{
    return o->hit_energy_fluct ? (double)FLT_MIN * 0x1p26 : (double)FLT_MIN;
}

}  // namespace

// ========================================================================
extern "C" {

void fcs_default_options(fcs_sim_options* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->mode = FCS_MODE_BATCHED;
    o->outputs = FCS_OUT_COMPACT;
    o->hit_energy_scale_mev = 100.0f;
    o->nhit_cap = 20000;
    o->min_layer_energy_mev = 1e-6;
    o->use_graph = 1;
}

const char* fcs_last_error(const fcs_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int fcs_create(fcs_ctx** out, int device)
{
    if (!out) return fail(nullptr, FCS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (device == FCS_DEVICE_NONE) {
        fcs_ctx* c = new fcs_ctx();
        c->dry = true;
        c->device = FCS_DEVICE_NONE;
        std::snprintf(c->name, sizeof c->name, "none");
        *out = c;
        return FCS_OK;
    }
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return fail(nullptr, FCS_E_NO_DEVICE, "no HIP device available");
    }
    if (device < 0 || device >= n)
        return fail(nullptr, FCS_E_NO_DEVICE, "device %d out of range [0, %d)", device, n);
    if (hipSetDevice(device) != hipSuccess) return fail(nullptr, FCS_E_HIP, "hipSetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return fail(nullptr, FCS_E_HIP, "hipGetDeviceProperties failed");
    if (prop.warpSize != 64)
        return fail(nullptr, FCS_E_NO_DEVICE, "device %d is not a wave64 device", device);
    fcs_ctx* c = new fcs_ctx();
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    std::snprintf(c->name, sizeof c->name, "%s", prop.gcnArchName);
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&c->ev_start) != hipSuccess || hipEventCreate(&c->ev_stop) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&c->ev_k0) != hipSuccess || hipEventCreate(&c->ev_k1) != hipSuccess ||
        hipEventCreate(&c->ev_p0) != hipSuccess || hipEventCreate(&c->ev_p1) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->win_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_loaded, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_spare_free, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_staged[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_staged[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_copied[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_copied[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_pre, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&c->h_ring, kRing * kBlockBytes) != hipSuccess) {
        fcs_destroy(c);
        return fail(nullptr, FCS_E_HIP, "stream/event/pinned allocation failed");
    }
    for (int i = 0; i < kRing; ++i)
        if (hipEventCreateWithFlags(&c->ring_ev[i], hipEventDisableTiming) != hipSuccess) {
            fcs_destroy(c);
            return fail(nullptr, FCS_E_HIP, "event creation failed");
        }
    for (int i = 0; i < kProfRing; ++i)
        if (hipEventCreate(&c->prof_ev[i][0]) != hipSuccess ||
            hipEventCreate(&c->prof_ev[i][1]) != hipSuccess) {
            fcs_destroy(c);
            return fail(nullptr, FCS_E_HIP, "event creation failed");
        }
    c->scratch = scratch_on_device(device);
    if (!c->scratch) {
        fcs_destroy(c);
        return fail(nullptr, FCS_E_HIP, "hipGetSymbolAddress of the scratch array failed");
    }
    if (ensure(c, c->w_params, kBlockBytes) ||
        ensure(c, c->w_queue, fcsk::kQueueInts * sizeof(int32_t)) ||
        ensure(c, c->w_async, sizeof(fcsk::AsyncAcc)) ||
        hipMemset(c->w_async.p, 0, sizeof(fcsk::AsyncAcc)) != hipSuccess) {
        fcs_destroy(c);
        return fail(nullptr, FCS_E_NOMEM, "device allocation failed");
    }
    *out = c;
    return FCS_OK;
}

void fcs_destroy(fcs_ctx* c)
{
    if (!c) return;
    if (c->dry) {
        delete c;
        return;
    }
    (void)hipSetDevice(c->device);
    if (c->copy_stream) (void)flush_host_copy(c);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->copy_stream) (void)hipStreamSynchronize(c->copy_stream);
    drop_graphs(c);
    c->q_valid = false;
    DevBuf* bufs[] = {&c->g_eta_lo, &c->g_eta_hi, &c->g_inv_deta, &c->g_inv_dphi, &c->g_phi_lo,
                      &c->g_neta, &c->g_nphi, &c->g_offset, &c->g_inv_r, &c->g_cell_id,
                      &c->p_e_edges, &c->p_eta_edges, &c->p_alpha, &c->p_weights, &c->p_cum,
                      &c->p_guide, &c->w_particles, &c->w_evoff, &c->w_override, &c->w_task_n,
                      &c->w_task_ehit, &c->w_part_ev, &c->w_part_p, &c->w_part_set,
                      &c->w_blk_sums, &c->w_blk_offs, &c->w_grp, &c->w_task_hoff, &c->w_chunks,
                      &c->w_small_rec, &c->w_tile_first, &c->w_cells, &c->g_layers, &c->g_regions,
                      &c->g_windows,
                      &c->w_flags, &c->w_seg_off, &c->w_seg_blk, &c->w_blk_list, &c->w_queue,
                      &c->w_params, &c->w_acc_el, &c->w_acc_bins, &c->w_hist_mark, &c->o_cells, &c->o_ids,
                      &c->o_e, &c->o_evoff, &c->o_heta, &c->o_hphi, &c->o_he, &c->o_hcell,
                      &c->o_thoff, &c->o_counts, &c->o_elayer, &c->w_async, &c->hs_ids[0],
                      &c->hs_ids[1], &c->hs_e[0], &c->hs_e[1], &c->hs_off[0], &c->hs_off[1],
                      &c->s_e_edges, &c->s_eta_edges, &c->s_alpha, &c->s_weights, &c->s_cum,
                      &c->s_guide};
    for (DevBuf* b : bufs) release(c, *b);
    if (c->h_ring) (void)hipHostFree(c->h_ring);
    if (c->h_tab) (void)hipHostFree(c->h_tab);
    if (c->ev_loaded) (void)hipEventDestroy(c->ev_loaded);
    if (c->ev_spare_free) (void)hipEventDestroy(c->ev_spare_free);
    for (int i = 0; i < kRing; ++i)
        if (c->ring_ev[i]) (void)hipEventDestroy(c->ring_ev[i]);
    for (int i = 0; i < kProfRing; ++i)
        for (int k = 0; k < 2; ++k)
            if (c->prof_ev[i][k]) (void)hipEventDestroy(c->prof_ev[i][k]);
    if (c->ev_done) (void)hipEventDestroy(c->ev_done);
    for (int i = 0; i < 2; ++i) {
        if (c->ev_staged[i]) (void)hipEventDestroy(c->ev_staged[i]);
        if (c->ev_copied[i]) (void)hipEventDestroy(c->ev_copied[i]);
    }
    if (c->ev_pre) (void)hipEventDestroy(c->ev_pre);
    if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
    if (c->win_stream) (void)hipStreamDestroy(c->win_stream);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->ev_start) (void)hipEventDestroy(c->ev_start);
    if (c->ev_stop) (void)hipEventDestroy(c->ev_stop);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_k0) (void)hipEventDestroy(c->ev_k0);
    if (c->ev_k1) (void)hipEventDestroy(c->ev_k1);
    if (c->ev_p0) (void)hipEventDestroy(c->ev_p0);
    if (c->ev_p1) (void)hipEventDestroy(c->ev_p1);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int fcs_get_info(const fcs_ctx* c, fcs_info* info)
{
    if (!c || !info) return FCS_E_INVALID_ARG;
    std::memset(info, 0, sizeof *info);
    std::snprintf(info->device_name, sizeof info->device_name, "%s", c->name);
    info->compute_units = c->n_cu;
    info->device = c->device;
    info->n_cells = c->has_geom ? c->n_cells : 0;
    info->n_layers = c->has_geom ? c->n_layers : 0;
    info->n_regions = c->has_geom ? c->n_regions : 0;
    info->n_histograms = c->has_param ? c->n_hist : 0;
    info->device_bytes = c->held;
    return FCS_OK;
}

int fcs_host_alloc(fcs_ctx* c, int64_t bytes, void** ptr)
{
    if (!c || !ptr) return FCS_E_INVALID_ARG;
    *ptr = nullptr;
    if (bytes < 1) return fail(c, FCS_E_INVALID_ARG, "bytes = %lld, must be >= 1", (long long)bytes);
    if (c->dry) return fail(c, FCS_E_NO_DEVICE, "context has no device");
    HIPCHK(c, hipSetDevice(c->device));
    if (hipHostMalloc(ptr, (size_t)bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        return fail(c, FCS_E_NOMEM, "pinned host allocation of %lld bytes failed", (long long)bytes);
    }
    return FCS_OK;
}

int fcs_host_free(fcs_ctx* c, void* ptr)
{
    if (!c) return FCS_E_INVALID_ARG;
    if (!ptr) return FCS_OK;
    if (c->dry) return fail(c, FCS_E_NO_DEVICE, "context has no device");
    HIPCHK(c, hipSetDevice(c->device));
    // the copy stream may still write into it
    int rc = flush_host_copy(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->copy_stream));
    HIPCHK(c, hipHostFree(ptr));
    return FCS_OK;
}

// ------------------------------------------------------------ geometry ---
int fcs_load_geometry(fcs_ctx* c, const fcs_geometry* g)
{
    const Range range("fcs_load_geometry");
    if (!c) return FCS_E_INVALID_ARG;
    if (!g) return fail(c, FCS_E_INVALID_ARG, "geometry is NULL");
    if (g->n_layers < 1 || g->n_layers > 64)
        return fail(c, FCS_E_INVALID_ARG, "n_layers = %d outside [1, 64]", g->n_layers);
    if (g->n_regions < 1 || g->n_regions > 8)
        return fail(c, FCS_E_INVALID_ARG, "n_regions = %d outside [1, 8]", g->n_regions);
    if (g->n_cells < 1 || g->n_cells > (1LL << 28))
        return fail(c, FCS_E_INVALID_ARG, "n_cells = %lld outside [1, 2^28]", (long long)g->n_cells);
    const void* ptrs[] = {g->cell_id, g->reg_eta_lo, g->reg_eta_hi, g->reg_inv_deta,
                          g->reg_inv_dphi, g->reg_phi_lo, g->reg_neta, g->reg_nphi,
                          g->reg_offset, g->layer_inv_r};
    const char* names[] = {"cell_id", "reg_eta_lo", "reg_eta_hi", "reg_inv_deta", "reg_inv_dphi",
                           "reg_phi_lo", "reg_neta", "reg_nphi", "reg_offset", "layer_inv_r"};
    for (int i = 0; i < 10; ++i)
        if (!ptrs[i]) return fail(c, FCS_E_INVALID_ARG, "geometry field %s is NULL", names[i]);
    const int L = g->n_layers, R = g->n_regions;
    long long run = 0;
    for (int l = 0; l < L; ++l) {
        if (!finite_pos(g->layer_inv_r[l]))
            return fail(c, FCS_E_INVALID_ARG, "layer_inv_r[%d] not finite and positive", l);
        for (int k = 0; k < R; ++k) {
            const int r = l * R + k;
            if (!std::isfinite(g->reg_eta_lo[r]) || !std::isfinite(g->reg_eta_hi[r]) ||
                !(g->reg_eta_lo[r] < g->reg_eta_hi[r]))
                return fail(c, FCS_E_INVALID_ARG, "reg_eta_lo/hi[%d] not an increasing range", r);
            if (k > 0 && g->reg_eta_lo[r] != g->reg_eta_hi[r - 1])
                return fail(c, FCS_E_INVALID_ARG, "region %d does not start where region %d ends",
                            r, r - 1);
            if (!finite_pos(g->reg_inv_deta[r]) || !finite_pos(g->reg_inv_dphi[r]) ||
                !std::isfinite(g->reg_phi_lo[r]))
                return fail(c, FCS_E_INVALID_ARG, "reg_inv_deta/inv_dphi/phi_lo[%d] invalid", r);
            if (g->reg_neta[r] < 1 || g->reg_nphi[r] < 1 || g->reg_neta[r] > 65535 ||
                g->reg_nphi[r] > 65535)
                return fail(c, FCS_E_INVALID_ARG, "reg_neta/nphi[%d] outside [1, 65535]", r);
            if (g->reg_offset[r] != run)
                return fail(c, FCS_E_INVALID_ARG, "reg_offset[%d] = %d, expected %lld", r,
                            g->reg_offset[r], run);
            run += (long long)g->reg_neta[r] * g->reg_nphi[r];
        }
    }
    if (run != g->n_cells)
        return fail(c, FCS_E_INVALID_ARG, "n_cells = %lld but regions hold %lld cells",
                    (long long)g->n_cells, run);
    if (c->dry) {
        c->n_cells = g->n_cells;
        c->n_layers = L;
        c->n_regions = R;
        c->has_geom = true;
        return FCS_OK;
    }
    HIPCHK(c, hipSetDevice(c->device));
    if (int rcf = flush_host_copy(c)) return rcf;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const size_t nr = (size_t)L * R;
    int rc = 0;
    if ((rc = upload(c, c->g_eta_lo, g->reg_eta_lo, nr)) || (rc = upload(c, c->g_eta_hi, g->reg_eta_hi, nr)) ||
        (rc = upload(c, c->g_inv_deta, g->reg_inv_deta, nr)) ||
        (rc = upload(c, c->g_inv_dphi, g->reg_inv_dphi, nr)) ||
        (rc = upload(c, c->g_phi_lo, g->reg_phi_lo, nr)) || (rc = upload(c, c->g_neta, g->reg_neta, nr)) ||
        (rc = upload(c, c->g_nphi, g->reg_nphi, nr)) || (rc = upload(c, c->g_offset, g->reg_offset, nr)) ||
        (rc = upload(c, c->g_inv_r, g->layer_inv_r, (size_t)L)) ||
        (rc = upload(c, c->g_cell_id, g->cell_id, (size_t)g->n_cells)))
        return rc;
    {
        // lookup records (see GeoLds): per layer (acc_lo, acc_hi, inv_r, -),
        // region lower edges 0..7 (+inf past the last); per region
        // (eta_lo, inv_deta, phi_lo, inv_dphi), (neta, nphi, offset, -)
        auto bits = [](float f) {
            int32_t v;
            std::memcpy(&v, &f, 4);
            return v;
        };
        const float inf = INFINITY;
        std::vector<int32_t> lay((size_t)L * 12, 0), reg((size_t)L * R * 8, 0);
        for (int l = 0; l < L; ++l) {
            int32_t* a = &lay[(size_t)l * 12];
            a[0] = bits(g->reg_eta_lo[l * R]);
            a[1] = bits(g->reg_eta_hi[l * R + R - 1]);
            a[2] = bits(g->layer_inv_r[l]);
            for (int k = 0; k < 8; ++k) a[4 + k] = bits(k < R ? g->reg_eta_lo[l * R + k] : inf);
            for (int k = 0; k < R; ++k) {
                int32_t* b = &reg[(size_t)(l * R + k) * 8];
                const int r = l * R + k;
                b[0] = bits(g->reg_eta_lo[r]);
                b[1] = bits(g->reg_inv_deta[r]);
                b[2] = bits(g->reg_phi_lo[r]);
                b[3] = bits(g->reg_inv_dphi[r]);
                b[4] = g->reg_neta[r];
                b[5] = g->reg_nphi[r];
                b[6] = g->reg_offset[r];
            }
        }
        if ((rc = upload(c, c->g_layers, lay.data(), lay.size())) ||
            (rc = upload(c, c->g_regions, reg.data(), reg.size())))
            return rc;
    }
    {
        // cell windows of the window pass: each layer's cells cut into runs
        // of at most kWinCells, each with the eta band its cells cover
        std::vector<int32_t> win;
        int nw = 0;
        for (int l = 0; l < L; ++l) {
            const long long lo = g->reg_offset[l * R];
            const long long hi = (long long)g->reg_offset[l * R + R - 1] +
                                 (long long)g->reg_neta[l * R + R - 1] * g->reg_nphi[l * R + R - 1];
            const int first = nw;
            const int n_l = (int)((hi - lo + fcsk::kWinCells - 1) / fcsk::kWinCells);
            for (int k = 0; k < n_l; ++k) {
                const long long c0 = lo + (long long)k * fcsk::kWinCells;
                const long long c1 = std::min(hi, c0 + fcsk::kWinCells);
                double b0 = INFINITY, b1 = -INFINITY;
                for (int q = 0; q < R; ++q) {
                    const int r = l * R + q;
                    const long long o0 = g->reg_offset[r];
                    const long long o1 = o0 + (long long)g->reg_neta[r] * g->reg_nphi[r];
                    if (o1 <= c0 || o0 >= c1) continue;
                    const long long ie0 = (std::max(c0, o0) - o0) / g->reg_nphi[r];
                    const long long ie1 = (std::min(c1, o1) - 1 - o0) / g->reg_nphi[r];
                    const double inv = (double)g->reg_inv_deta[r];
                    b0 = std::min(b0, (double)g->reg_eta_lo[r] + (double)ie0 / inv);
                    b1 = std::max(b1, (double)g->reg_eta_lo[r] + (double)(ie1 + 1) / inv);
                }
                const float f0 = (float)b0, f1 = (float)b1;
                int32_t b0i, b1i;
                std::memcpy(&b0i, &f0, 4);
                std::memcpy(&b1i, &f1, 4);
                const int32_t rec[8] = {l, (int32_t)c0, (int32_t)c1, first, b0i, b1i, n_l, 0};
                win.insert(win.end(), rec, rec + 8);
                ++nw;
            }
        }
        c->n_windows = nw <= kMaxWindows ? nw : 0;  // very fine geometries: no window pass
        if (c->n_windows && (rc = upload(c, c->g_windows, win.data(), win.size()))) return rc;
    }
    const bool changed = !c->has_geom || c->n_cells != g->n_cells;
    c->n_cells = g->n_cells;
    c->n_layers = L;
    c->n_regions = R;
    c->has_geom = true;
    // Captured launch sequences hold grids and LDS sizes derived from the
    // layer and region counts, and a kept work queue holds the old layout:
    // neither survives a reload.
    drop_graphs(c);
    c->q_valid = false;
    if (changed) {
        // accumulator layout depends on the cell count: start it over
        release(c, c->w_cells);
        release(c, c->w_flags);
        c->cells_events = 0;
        c->flag_events = 0;
    }
    if (c->has_param && c->n_layers != L) c->has_param = false;
    // tables loading asynchronously for another layer count are not used
    if (c->pending && c->s_hist != 3LL * c->s_ebins * c->s_etabins * L) c->pending = false;
    return FCS_OK;
}

// ------------------------------------------------------ parametrization ---
}  // extern "C"

namespace {

// host-side checks of a parametrization; *n_hist receives its histogram count
int check_param(fcs_ctx* c, const fcs_param* p, long long* n_hist_out)
{
    if (!p) return fail(c, FCS_E_INVALID_ARG, "param is NULL");
    if (!c->has_geom) return fail(c, FCS_E_NOT_LOADED, "load the geometry first");
    if (p->n_types != 3) return fail(c, FCS_E_INVALID_ARG, "n_types = %d, must be 3", p->n_types);
    if (p->n_ebins < 1 || p->n_ebins > 64 || p->n_etabins < 1 || p->n_etabins > 64)
        return fail(c, FCS_E_INVALID_ARG, "n_ebins / n_etabins outside [1, 64]");
    if (p->n_layers != c->n_layers)
        return fail(c, FCS_E_INVALID_ARG, "n_layers = %d but the geometry has %d", p->n_layers,
                    c->n_layers);
    if (p->n_rbins != 32 || p->n_abins != 8)
        return fail(c, FCS_E_INVALID_ARG, "histograms must be 32 (r) x 8 (alpha) bins");
    if (!finite_pos(p->r_max_mm)) return fail(c, FCS_E_INVALID_ARG, "r_max_mm not finite and positive");
    if (!p->e_edges || !p->eta_edges || !p->dirichlet_alpha || !p->weights)
        return fail(c, FCS_E_INVALID_ARG, "e_edges, eta_edges, dirichlet_alpha and weights are required");
    for (int k = 0; k <= p->n_ebins; ++k)
        if (!std::isfinite(p->e_edges[k]) || (k > 0 && !(p->e_edges[k] > p->e_edges[k - 1])))
            return fail(c, FCS_E_INVALID_ARG, "e_edges not finite and increasing at %d", k);
    for (int k = 0; k <= p->n_etabins; ++k)
        if (!std::isfinite(p->eta_edges[k]) || (k > 0 && !(p->eta_edges[k] > p->eta_edges[k - 1])))
            return fail(c, FCS_E_INVALID_ARG, "eta_edges not finite and increasing at %d", k);
    const int L = p->n_layers;
    for (int i = 0; i < 3 * L; ++i)
        if (!finite_pos(p->dirichlet_alpha[i]))
            return fail(c, FCS_E_INVALID_ARG, "dirichlet_alpha[%d] not finite and positive", i);
    const long long n_hist = 3LL * p->n_ebins * p->n_etabins * L;
    // weights finite and >= 0, and at least one positive per histogram (then
    // its FP64 total is positive); branch-free per histogram so that the
    // loop vectorizes (tables at full-sample volume hold ~10^8 weights)
    for (long long h = 0; h < n_hist; ++h) {
        const float* wh = p->weights + h * 256;
        int bad = 0, pos = 0;
        for (int b = 0; b < 256; ++b) {
            const float w = wh[b];
            bad |= !(w >= 0.f && w <= FLT_MAX);
            pos |= w > 0.f;
        }
        if (bad) {
            int b = 0;
            while (wh[b] >= 0.f && wh[b] <= FLT_MAX) ++b;
            return fail(c, FCS_E_INVALID_ARG, "weights[%lld] negative or not finite", h * 256 + b);
        }
        if (!pos) return fail(c, FCS_E_INVALID_ARG, "histogram %lld has no weight", h);
    }
    *n_hist_out = n_hist;
    return FCS_OK;
}

// Switch to the tables of a finished-or-running asynchronous load: the
// context's stream waits for it (no host wait), the second set becomes the
// one calls use, the former one is the spare.  Called by every call that
// enqueues work reading the tables.
int activate_tables(fcs_ctx* c)
{
    if (!c->pending) return FCS_OK;
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_loaded, 0));
    std::swap(c->p_e_edges, c->s_e_edges);
    std::swap(c->p_eta_edges, c->s_eta_edges);
    std::swap(c->p_alpha, c->s_alpha);
    std::swap(c->p_weights, c->s_weights);
    std::swap(c->p_cum, c->s_cum);
    std::swap(c->p_guide, c->s_guide);
    std::swap(c->n_types, c->s_types);
    std::swap(c->n_ebins, c->s_ebins);
    std::swap(c->n_etabins, c->s_etabins);
    std::swap(c->r_max, c->s_rmax);
    std::swap(c->n_hist, c->s_hist);
    c->pending = false;
    c->has_param = true;
    c->q_valid = false;  // a kept work queue refers to the former tables
    // the former set is the spare now; the calls enqueued so far may read it
    HIPCHK(c, hipEventRecord(c->ev_spare_free, c->stream));
    return FCS_OK;
}

}  // namespace

extern "C" {

int fcs_load_parametrization(fcs_ctx* c, const fcs_param* p)
{
    const Range range("fcs_load_parametrization");
    if (!c) return FCS_E_INVALID_ARG;
    long long n_hist = 0;
    int rc = check_param(c, p, &n_hist);
    if (rc) return rc;
    const int L = p->n_layers;
    if (c->dry) {
        c->n_types = p->n_types;
        c->n_ebins = p->n_ebins;
        c->n_etabins = p->n_etabins;
        c->r_max = p->r_max_mm;
        c->n_hist = n_hist;
        c->has_param = true;
        return FCS_OK;
    }
    HIPCHK(c, hipSetDevice(c->device));
    if (int rcf = flush_host_copy(c)) return rcf;
    // this load supersedes an asynchronous one not yet taken into use
    if (c->load_in_flight) HIPCHK(c, hipEventSynchronize(c->ev_loaded));
    c->pending = false;
    c->load_in_flight = false;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // a kept work queue refers to the old tables (their pointers and
    // histogram count): an adjoint may not reuse it after a reload
    c->q_valid = false;
    if ((rc = upload(c, c->p_e_edges, p->e_edges, (size_t)p->n_ebins + 1)) ||
        (rc = upload(c, c->p_eta_edges, p->eta_edges, (size_t)p->n_etabins + 1)) ||
        (rc = upload(c, c->p_alpha, p->dirichlet_alpha, (size_t)3 * L)) ||
        (rc = upload(c, c->p_weights, p->weights, (size_t)n_hist * 256)) ||
        (rc = ensure(c, c->p_cum, (size_t)n_hist * 256 * sizeof(float))) ||
        (rc = ensure(c, c->p_guide, (size_t)n_hist * fcsk::kGuide)))
        return rc;
    hipLaunchKernelGGL(fcsk::k_build_cum, dim3(grid_for(n_hist, fcsk::kCumHist)), dim3(fcsk::kCumHist), 0, c->stream,
                       (const float*)c->p_weights.p, (float*)c->p_cum.p, n_hist);
    hipLaunchKernelGGL(fcsk::k_build_guide, dim3(grid_for(n_hist, fcsk::kBlock / fcsk::kWave)), dim3(fcsk::kBlock), 0,
                       c->stream, (const float*)c->p_cum.p, (uint8_t*)c->p_guide.p, n_hist);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->n_types = p->n_types;
    c->n_ebins = p->n_ebins;
    c->n_etabins = p->n_etabins;
    c->r_max = p->r_max_mm;
    c->n_hist = n_hist;
    c->has_param = true;
    return FCS_OK;
}

int fcs_load_parametrization_async(fcs_ctx* c, const fcs_param* p)
{
    const Range range("fcs_load_parametrization_async");
    if (!c) return FCS_E_INVALID_ARG;
    long long n_hist = 0;
    int rc = check_param(c, p, &n_hist);
    if (rc) return rc;
    if (c->dry) return fcs_load_parametrization(c, p);
    const int L = p->n_layers;
    HIPCHK(c, hipSetDevice(c->device));
    if (int rcf = flush_host_copy(c)) return rcf;
    // a load not yet taken into use is taken into use now: this one goes to
    // the set it replaces
    if ((rc = activate_tables(c))) return rc;
    // the spare set may still be read by the calls enqueued before it was
    // retired (ev_spare_free), and the pinned staging by the previous load's
    // copies
    if (c->load_in_flight) HIPCHK(c, hipEventSynchronize(c->ev_loaded));
    const size_t b_e = (size_t)(p->n_ebins + 1) * 4, b_h = (size_t)(p->n_etabins + 1) * 4,
                 b_a = (size_t)3 * L * 4, b_w = (size_t)n_hist * 256 * 4;
    const size_t o_h = (b_e + 255) & ~(size_t)255, o_a = o_h + ((b_h + 255) & ~(size_t)255),
                 o_w = o_a + ((b_a + 255) & ~(size_t)255), need = o_w + b_w;
    if (c->h_tab_bytes < need) {
        if (c->h_tab) HIPCHK(c, hipHostFree(c->h_tab));
        c->h_tab = nullptr;
        c->h_tab_bytes = 0;
        if (hipHostMalloc((void**)&c->h_tab, need, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            c->h_tab = nullptr;
            return fail(c, FCS_E_NOMEM, "pinned staging of %zu bytes failed", need);
        }
        c->h_tab_bytes = need;
    }
    std::memcpy(c->h_tab, p->e_edges, b_e);
    std::memcpy(c->h_tab + o_h, p->eta_edges, b_h);
    std::memcpy(c->h_tab + o_a, p->dirichlet_alpha, b_a);
    std::memcpy(c->h_tab + o_w, p->weights, b_w);
    // growing the spare set frees its old buffers: wait for the calls that
    // may read them
    const bool grow = c->s_weights.bytes < b_w || c->s_cum.bytes < b_w ||
                      c->s_guide.bytes < (size_t)n_hist * fcsk::kGuide || c->s_e_edges.bytes < b_e ||
                      c->s_eta_edges.bytes < b_h || c->s_alpha.bytes < b_a;
    if (grow) HIPCHK(c, hipEventSynchronize(c->ev_spare_free));
    if ((rc = ensure(c, c->s_e_edges, b_e)) || (rc = ensure(c, c->s_eta_edges, b_h)) ||
        (rc = ensure(c, c->s_alpha, b_a)) || (rc = ensure(c, c->s_weights, b_w)) ||
        (rc = ensure(c, c->s_cum, b_w)) || (rc = ensure(c, c->s_guide, (size_t)n_hist * fcsk::kGuide)))
        return rc;
    hipStream_t cs = c->copy_stream;
    HIPCHK(c, hipStreamWaitEvent(cs, c->ev_spare_free, 0));
    HIPCHK(c, hipMemcpyAsync(c->s_e_edges.p, c->h_tab, b_e, hipMemcpyHostToDevice, cs));
    HIPCHK(c, hipMemcpyAsync(c->s_eta_edges.p, c->h_tab + o_h, b_h, hipMemcpyHostToDevice, cs));
    HIPCHK(c, hipMemcpyAsync(c->s_alpha.p, c->h_tab + o_a, b_a, hipMemcpyHostToDevice, cs));
    HIPCHK(c, hipMemcpyAsync(c->s_weights.p, c->h_tab + o_w, b_w, hipMemcpyHostToDevice, cs));
    hipLaunchKernelGGL(fcsk::k_build_cum, dim3(grid_for(n_hist, fcsk::kCumHist)), dim3(fcsk::kCumHist), 0, cs,
                       (const float*)c->s_weights.p, (float*)c->s_cum.p, n_hist);
    hipLaunchKernelGGL(fcsk::k_build_guide, dim3(grid_for(n_hist, fcsk::kBlock / fcsk::kWave)), dim3(fcsk::kBlock), 0, cs,
                       (const float*)c->s_cum.p, (uint8_t*)c->s_guide.p, n_hist);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipEventRecord(c->ev_loaded, cs));
    c->s_types = p->n_types;
    c->s_ebins = p->n_ebins;
    c->s_etabins = p->n_etabins;
    c->s_rmax = p->r_max_mm;
    c->s_hist = n_hist;
    c->pending = true;
    c->load_in_flight = true;
    return FCS_OK;
}

}  // extern "C"

// ================================================================ batch ===
namespace {

struct Shape {
    long long n_particles, part_base, n_events, ev0;
    long long hit_base, out_base;
};

struct Tuning {
    int chunk, big, tile, wg_per_cu, win_parts;
};

int check_tuning(fcs_ctx* c, const fcs_sim_options* o, Tuning* t)
{
    t->chunk = o->chunk_hits ? o->chunk_hits : 2048;
    t->big = o->big_task_hits ? o->big_task_hits : 128;
    t->tile = o->tile_hits ? o->tile_hits : 512;
    t->wg_per_cu = o->wg_per_cu ? o->wg_per_cu : 4;
    t->win_parts = o->window_particles ? o->window_particles : 1024;
    if (t->win_parts < 64 || t->win_parts > 65536)
        return fail(c, FCS_E_INVALID_ARG, "window_particles = %d outside [64, 65536]", t->win_parts);
    if (o->window_pass < -1 || o->window_pass > 1)
        return fail(c, FCS_E_INVALID_ARG, "window_pass = %d: use -1, 0 or 1", o->window_pass);
    if (o->host_copy_workgroups < -1 || o->host_copy_workgroups > 4096)
        return fail(c, FCS_E_INVALID_ARG, "host_copy_workgroups = %d outside [-1, 4096]",
                    o->host_copy_workgroups);
    if (t->chunk < 1 || t->chunk > fcsk::kChunkMax)
        return fail(c, FCS_E_INVALID_ARG, "chunk_hits = %d outside [1, %d]", t->chunk, fcsk::kChunkMax);
    if (t->tile < fcsk::kWave || t->tile > fcsk::kTileMax || t->tile % fcsk::kWave)
        return fail(c, FCS_E_INVALID_ARG, "tile_hits = %d must be a multiple of 64 in [64, %d]",
                    t->tile, fcsk::kTileMax);
    if (t->big < 1 || t->big > t->tile)
        return fail(c, FCS_E_INVALID_ARG, "big_task_hits = %d outside [1, tile_hits]", t->big);
    if (t->wg_per_cu < 1 || t->wg_per_cu > 32)
        return fail(c, FCS_E_INVALID_ARG, "wg_per_cu = %d outside [1, 32]", t->wg_per_cu);
    return FCS_OK;
}

// the inputs and options a work queue is built from (device inputs)
fcs_ctx::QueueKey queue_key(const fcs_sim_options* o, const Tuning& tu, const void* particles,
                            const void* evoff, long long n_events, long long N, long long ev_base)
{
    fcs_ctx::QueueKey k{};
    k.particles = particles;
    k.evoff = evoff;
    k.override_ = o->elayer_override;
    k.n_events = n_events;
    k.n_particles = N;
    k.ev_base = ev_base;
    k.seed = o->seed;
    k.scale = o->hit_energy_scale_mev;
    k.cap = o->nhit_cap;
    k.min_e = o->min_layer_energy_mev;
    k.chunk = tu.chunk;
    k.big = tu.big;
    k.tile = tu.tile;
    return k;
}

// Fill the Params block for one launch sequence over a range of events.

// scan blocks (kBlock / L particles each) per setup workgroup: as many as
// fit (longer task lists per lane), while the batch still gives about four
// workgroups per CU
int setup_sub(long long N, int L, int n_cu)
{
    const long long ppb = fcsk::kBlock / L;
    const long long fill = N / (ppb * 4LL * n_cu);
    const long long cap = std::min<long long>(fcsk::kSetupSubMax, std::max<long long>(1, fcsk::kSetupPartCap / ppb));
    return (int)std::max<long long>(1, std::min(cap, fill));
}
// the setup launch of a batch of N particles: one scan block per workgroup
// (k_setup_one), or setup_sub of them (k_setup)
void launch_setup(hipStream_t s, const Params* dP, long long N, int L, int n_cu)
{
    const int sub = setup_sub(N, L, n_cu);
    if (sub == 1)
        hipLaunchKernelGGL(fcsk::k_setup_one, dim3(grid_for(N, fcsk::kBlock / L)), dim3(fcsk::kBlock), 0, s, dP);
    else
        hipLaunchKernelGGL(fcsk::k_setup, dim3(grid_for(N, (fcsk::kBlock / L) * sub)), dim3(fcsk::kBlock), 0, s,
                           dP);
}

// Where a call's workspace lives: the context's grow-only buffers, or (with
// `base`, no-allocation calls) consecutive 256-byte aligned pieces of the
// scratch array, in the order they are taken.
struct Carver {
    fcs_ctx* c;
    char* base;
    size_t used;
    int take(DevBuf& b, size_t bytes, void** out, bool* grown = nullptr)
    {
        if (!base) {
            const int rc = ensure(c, b, bytes, grown);
            *out = b.p;
            return rc;
        }
        bytes = bytes ? (bytes + 255) & ~(size_t)255 : 256;
        if (used + bytes > kScratchBytes)
            return fail(c, FCS_E_INVALID_ARG,
                        "batch too large for fcs_simulate_events_noalloc: its workspace needs more "
                        "than the %zu bytes of the scratch array (split the batch)", kScratchBytes);
        *out = base + used;
        used += bytes;
        return FCS_OK;
    }
    size_t left() const { return base ? kScratchBytes - used : 0; }
};

// `dense_out` (device) is the caller's dense cell buffer or NULL.  With
// `scratch` (the device's scratch array) nothing is allocated: the whole
// workspace, the parameter block and the tickets are carved from it, the
// block counts and the private accumulator are zeroed by the call itself,
// and the chunk list takes what remains of the array.
int prepare(fcs_ctx* c, const fcs_sim_options* o, const Tuning& tu, const Shape& sh,
            const fcsk::Particle* d_particles, const long long* d_evoff, const float* d_override,
            float* dense_out, const fcs_sim_output* dout, bool want_hits, bool async, Params* P,
            char* scratch = nullptr, bool allow_win = false)
{
    const int L = c->n_layers;
    const long long N = sh.n_particles;
    const long long nt = N * L;
    const long long E = sh.n_events;
    // flag stride per event: the 64-cell blocks rounded up to whole segments
    // and then to a power of two, so that (event, block) packs into 32 bits
    const int n_seg = (int)(((c->n_cells + 63) / 64 + fcsk::kSegBlocks - 1) / fcsk::kSegBlocks);
    int blk_shift = 0;
    while ((1 << blk_shift) < n_seg * fcsk::kSegBlocks) ++blk_shift;
    const int n_blk = 1 << blk_shift;
    if ((sh.n_events << blk_shift) > 0xffffffffLL)
        return fail(c, FCS_E_INVALID_ARG, "%lld events in one batch: at most %lld for this geometry",
                    (long long)sh.n_events, 0xffffffffLL >> blk_shift);
    // the task scan runs over the setup blocks (kBlock / L particles each)
    const long long nsb = (N + fcsk::kBlock / L - 1) / (fcsk::kBlock / L);
    const long long nsg = (nsb + fcsk::kGroupItems - 1) / fcsk::kGroupItems;
    const long long nseg = E * n_seg;
    const long long nsegb = (nseg + fcsk::kSegGroup - 1) / fcsk::kSegGroup;
    if (c->chunk_cap < nt + 1024) c->chunk_cap = nt + 1024;
    // an asynchronous call cannot retry with a larger chunk list: reserve
    // the most chunks the hit cap allows
    if (async) {
        const long long most = nt * ((o->nhit_cap + tu.chunk - 1) / tu.chunk) + 1024;
        if (c->chunk_cap < most) c->chunk_cap = most;
    }
    int rc = 0;
    Carver cv{c, scratch, 0};
    void *p_params = nullptr, *p_queue = nullptr, *p_task_n, *p_task_ehit, *p_part_ev, *p_part_p,
         *p_part_set, *p_blk_sums, *p_blk_offs, *p_grp, *p_task_hoff, *p_small_rec, *p_tile_first,
         *p_seg_off, *p_seg_blk, *p_blk_list, *p_flags, *p_cells = nullptr, *p_chunks;
    if (scratch) {
        // the parameter block first (kernels and uploads address it), then
        // the tickets, then the buffers that must start at zero
        if ((rc = cv.take(c->w_params, kBlockBytes, &p_params)) ||
            (rc = cv.take(c->w_queue, fcsk::kQueueInts * sizeof(int32_t), &p_queue)) ||
            (rc = cv.take(c->w_flags, (size_t)E * n_blk, &p_flags)) ||
            (!dense_out && (rc = cv.take(c->w_cells, (size_t)E * c->n_cells * 4, &p_cells))))
            return rc;
    } else {
        p_params = c->w_params.p;
        p_queue = c->w_queue.p;
    }
    if ((rc = cv.take(c->w_task_n, nt * 4, &p_task_n)) || (rc = cv.take(c->w_task_ehit, nt * 4, &p_task_ehit)) ||
        (rc = cv.take(c->w_part_ev, N * 4, &p_part_ev)) || (rc = cv.take(c->w_part_p, N * 4, &p_part_p)) ||
        (rc = cv.take(c->w_part_set, N * 4, &p_part_set)) ||
        (rc = cv.take(c->w_blk_sums, nsb * 16, &p_blk_sums)) ||
        (rc = cv.take(c->w_blk_offs, nsb * 16, &p_blk_offs)) || (rc = cv.take(c->w_grp, nsg * 40, &p_grp)) ||
        (rc = cv.take(c->w_task_hoff, want_hits ? nt * 4 : 4, &p_task_hoff)) ||
        (rc = cv.take(c->w_small_rec, (size_t)nt * 32, &p_small_rec)) ||
        (rc = cv.take(c->w_tile_first, (nt + 1) * 4, &p_tile_first)) ||
        (rc = cv.take(c->w_seg_off, nseg * 8, &p_seg_off)) ||
        (rc = cv.take(c->w_seg_blk, nsegb * 8, &p_seg_blk)) ||
        (rc = cv.take(c->w_blk_list, (size_t)nseg * fcsk::kSegBlocks * 8, &p_blk_list)))
        return rc;
    long long chunk_cap = c->chunk_cap;
    if (scratch) {
        // the chunk list takes the rest of the array; a batch needing more
        // chunks than that fails (the call cannot grow it)
        chunk_cap = std::min<long long>((long long)(cv.left() / 16), 2147483647LL);
        if (chunk_cap < 1024)
            return fail(c, FCS_E_INVALID_ARG,
                        "batch too large for fcs_simulate_events_noalloc: no room left for its work "
                        "queue in the %zu-byte scratch array (split the batch)", kScratchBytes);
        p_chunks = scratch + cv.used;
        // what must start at zero: the block counts and the accumulator
        hipLaunchKernelGGL(fcsk::k_fill_u8, dim3(1024), dim3(256), 0, c->stream, (uint8_t*)p_flags,
                           (long long)E * n_blk);
        if (p_cells)
            hipLaunchKernelGGL(fcsk::k_fill_u32, dim3(4096), dim3(256), 0, c->stream, (uint32_t*)p_cells,
                               E * c->n_cells, 0u);
    } else {
        if ((rc = cv.take(c->w_chunks, (size_t)chunk_cap * 16, &p_chunks))) return rc;
        // flags and the private accumulator are kept zero between calls
        if (c->flag_events < E) {
            if ((rc = ensure(c, c->w_flags, (size_t)E * n_blk))) return rc;
            hipLaunchKernelGGL(fcsk::k_fill_u8, dim3(1024), dim3(256), 0, c->stream,
                               (uint8_t*)c->w_flags.p, (long long)(c->w_flags.bytes));
            c->flag_events = (long long)(c->w_flags.bytes / (size_t)n_blk);
        }
        p_flags = c->w_flags.p;
        if (!dense_out && c->cells_events < E) {
            if ((rc = ensure(c, c->w_cells, (size_t)E * c->n_cells * 4))) return rc;
            hipLaunchKernelGGL(fcsk::k_fill_u32, dim3(4096), dim3(256), 0, c->stream,
                               (uint32_t*)c->w_cells.p, (long long)(c->w_cells.bytes / 4), 0u);
            c->cells_events = (long long)(c->w_cells.bytes / 4 / (size_t)c->n_cells);
        }
        if (!dense_out) p_cells = c->w_cells.p;
    }
    HIPCHK(c, hipGetLastError());
    c->cur_params = (char*)p_params;

    std::memset(P, 0, sizeof *P);
    P->n_cells = c->n_cells;
    P->n_layers = L;
    P->n_regions = c->n_regions;
    P->n_blk = n_blk;
    P->blk_shift = blk_shift;
    P->n_seg = n_seg;
    P->reg_eta_lo = (const float*)c->g_eta_lo.p;
    P->reg_eta_hi = (const float*)c->g_eta_hi.p;
    P->reg_inv_deta = (const float*)c->g_inv_deta.p;
    P->reg_inv_dphi = (const float*)c->g_inv_dphi.p;
    P->reg_phi_lo = (const float*)c->g_phi_lo.p;
    P->reg_neta = (const int32_t*)c->g_neta.p;
    P->reg_nphi = (const int32_t*)c->g_nphi.p;
    P->reg_offset = (const int32_t*)c->g_offset.p;
    P->layer_inv_r = (const float*)c->g_inv_r.p;
    P->cell_id = (const long long*)c->g_cell_id.p;
    P->n_types = c->n_types;
    P->n_ebins = c->n_ebins;
    P->n_etabins = c->n_etabins;
    P->r_max = c->r_max;
    P->e_edges = (const float*)c->p_e_edges.p;
    P->eta_edges = (const float*)c->p_eta_edges.p;
    P->alpha = (const float*)c->p_alpha.p;
    P->cum = (const float*)c->p_cum.p;
    P->guide = (const uint8_t*)c->p_guide.p;
    P->weights = (const float*)c->p_weights.p;
    P->n_hist = c->n_hist;
    P->key0 = (uint32_t)(o->seed & 0xffffffffu);
    P->key1 = (uint32_t)(o->seed >> 32);
    P->ev_base = o->event_index_base + (unsigned long long)sh.ev0;
    P->n_particles = N;
    P->part_base = sh.part_base;
    P->n_events = E;
    P->n_tasks = nt;
    P->particles = d_particles;
    P->ev_off = d_evoff;
    P->elayer_override = d_override;
    P->scale = o->hit_energy_scale_mev;
    P->cap = o->nhit_cap;
    P->min_e = o->min_layer_energy_mev;
    P->ehit_min = (float)min_hit_energy(o);
    P->placement_f64 = o->placement_fp64 ? 1 : 0;
    P->hit_fluct = o->hit_energy_fluct ? 1 : 0;
    P->chunk_hits = tu.chunk;
    P->big_thr = tu.big;
    P->tile_hits = tu.tile;
    P->want_hits = want_hits ? 1 : 0;
    P->clean_cells = dense_out ? 0 : 1;
    P->chunk_cap = (int)std::min<long long>(chunk_cap, 2147483647LL);
    P->n_scan_blocks = (int)nsb;
    P->n_scan_groups = (int)nsg;
    P->setup_sub = setup_sub(N, L, c->n_cu);
    P->n_seg_groups = (int)nsegb;
    P->task_n = (int32_t*)p_task_n;
    P->task_ehit = (float*)p_task_ehit;
    P->part_ev = (int32_t*)p_part_ev;
    P->part_p = (uint32_t*)p_part_p;
    P->part_set = (int32_t*)p_part_set;
    P->blk_sums = (int32_t*)p_blk_sums;
    P->blk_offs = (int32_t*)p_blk_offs;
    // group records: rest and offsets (16 bytes each, aligned), then hits
    P->grp_rest = (int32_t*)p_grp;
    P->grp_offs = (int32_t*)((char*)p_grp + nsg * 16);
    P->grp_hits = (long long*)((char*)p_grp + nsg * 32);
    P->task_hoff = (int32_t*)p_task_hoff;
    P->chunks = (int4*)p_chunks;
    P->small_rec = (int4*)p_small_rec;
    P->geo_layers = (const int4*)c->g_layers.p;
    P->geo_regions = (const int4*)c->g_regions.p;
    P->tile_first = (int32_t*)p_tile_first;
    P->cells = dense_out ? dense_out : (float*)p_cells;
    P->flags = (uint8_t*)p_flags;
    P->seg_off = (long long*)p_seg_off;
    P->seg_blk = (long long*)p_seg_blk;
    P->blk_list = (unsigned long long*)p_blk_list;
    P->ctr = (Counters*)((char*)p_params + kCtrOffset);
    P->queue = (int32_t*)p_queue;
    if (dout) {
        P->out_elayer = dout->elayer;
        P->out_counts = dout->counts;
        P->out_ids = (long long*)dout->cell_ids;
        P->out_e = dout->cell_e;
        P->out_cap = dout->cell_ids ? dout->cell_capacity : 0;
        P->out_ev_off = (long long*)dout->event_cell_offsets;
        P->hit_eta = dout->hit_eta;
        P->hit_phi = dout->hit_phi;
        P->hit_e = dout->hit_e;
        P->hit_cell = dout->hit_cell;
        P->hit_cap = want_hits ? dout->hit_capacity : 0;
        P->out_task_hoff = (long long*)dout->task_hit_offsets;
    }
    P->hit_base = sh.hit_base;
    P->out_base = sh.out_base;
    // the window pass (small tasks of many-particle events by cell windows)
    const bool dense_events = sh.n_particles >= kWinMinParticlesPerEvent * sh.n_events;
    P->win_path = allow_win && c->n_windows > 0 && !o->placement_fp64 && !o->hit_energy_fluct &&
                  (o->window_pass == 1 || (o->window_pass == 0 && dense_events)) ? 1 : 0;
    P->win_parts = tu.win_parts;
    P->n_windows = c->n_windows;
    P->geo_windows = (const int4*)c->g_windows.p;
    // the window pass has no small-task records: their buffer holds the
    // layer-major (hits, Ehit) pairs it reads instead
    P->task_nT = P->win_path ? (unsigned long long*)P->small_rec : nullptr;
    return FCS_OK;
}

// LDS bytes of the geometry records the hit kernels stage
size_t geo_lds_bytes(const Params& P) { return (size_t)(3 * P.n_layers + 2 * P.n_layers * P.n_regions) * 16; }

// Enqueue the launch sequence of one batch on c->stream (the window pass
// may fork onto win_stream and join back within the same part).  All
// kernels read the device Params block, so a sequence can be captured once
// and replayed.  part: 0 = everything, 1 = the setup pass (with the task
// scans unless they run beside the window pass), 2 = the hit step: window
// pass and hit kernel (with the scans beside the window pass when it forks),
// 3 = compaction and reset.
enum Part { kAll = 0, kPre = 1, kHits = 2, kPost = 3 };
// where the cell energies go: the private accumulator (compacted, then
// cleared), the caller's dense buffer and the compacted list, or the
// caller's dense buffer alone (no compaction; the block counts are cleared)
enum CellMode { kPrivate = 0, kDenseCompact = 1, kDenseOnly = 2 };

void enqueue_batch(fcs_ctx* c, const Params& P, int mode, int grid, int part)
{
    const bool dense = mode != kPrivate;
    const Params* dP = (const Params*)c->cur_params;
    hipStream_t s = c->stream;
    // the window pass needs the setup pass's outputs only (and the task
    // scans' hit offsets when it writes hit lists): it then runs on the
    // second stream beside the scans, which open the hit step
    const bool fork = P.win_path && !P.want_hits;
    const auto scans = [&]() {
        hipLaunchKernelGGL(fcsk::k_scan_group, dim3(P.n_scan_groups), dim3(fcsk::kScanThreads), 0, s, dP);
        if (P.n_scan_groups > 1)
            hipLaunchKernelGGL(fcsk::k_scan_top, dim3(1), dim3(fcsk::kScanThreads), 0, s, dP);
        hipLaunchKernelGGL(fcsk::k_scan_write, dim3(P.n_scan_blocks), dim3(fcsk::kBlock), 0, s, dP);
    };
    const auto windows = [&](hipStream_t ws) {
        hipLaunchKernelGGL(fcsk::k_windows, dim3(c->n_cu * fcsk::kWinPerCu), dim3(fcsk::kWinThreads),
                           geo_lds_bytes(P) + (size_t)P.n_windows * 32, ws, dP);
    };
    if (part == kAll || part == kPre) {
        if (dense) hipLaunchKernelGGL(fcsk::k_fill_dense, dim3(2048), dim3(256), 0, s, dP);
        launch_setup(s, dP, P.n_particles, P.n_layers, c->n_cu);
        if (!fork) scans();
    }
    if ((part == kAll || part == kHits) && fork) {
        (void)hipEventRecord(c->ev_fork, s);
        (void)hipStreamWaitEvent(c->win_stream, c->ev_fork, 0);
        windows(c->win_stream);
        (void)hipEventRecord(c->ev_join, c->win_stream);
        scans();
    } else if ((part == kAll || part == kHits) && P.win_path) {
        windows(s);
    }
    if ((part == kAll || part == kHits) && P.placement_f64)
        hipLaunchKernelGGL((fcsk::k_hits<true, false>), dim3(grid), dim3(fcsk::kBlock), geo_lds_bytes(P), s, dP);
    else if ((part == kAll || part == kHits) && P.hit_fluct)
        hipLaunchKernelGGL((fcsk::k_hits<false, true>), dim3(grid), dim3(fcsk::kBlock), geo_lds_bytes(P), s, dP);
    else if ((part == kAll || part == kHits) && P.win_path)
        hipLaunchKernelGGL((fcsk::k_hits<false, false, false>), dim3(grid), dim3(fcsk::kBlock), geo_lds_bytes(P), s,
                           dP);
    else if (part == kAll || part == kHits)
        hipLaunchKernelGGL((fcsk::k_hits<false, false>), dim3(grid), dim3(fcsk::kBlock), geo_lds_bytes(P), s, dP);
    if ((part == kAll || part == kHits) && fork) (void)hipStreamWaitEvent(s, c->ev_join, 0);
    if ((part == kAll || part == kPost) && mode == kDenseOnly) {
        const long long words = P.n_events << (P.blk_shift - 4);
        hipLaunchKernelGGL(fcsk::k_flags_reset,
                           dim3((unsigned)std::min<long long>(grid_for(words, fcsk::kBlock), (long long)c->n_cu * 8)),
                           dim3(fcsk::kBlock), 0, s, dP);
    } else if (part == kAll || part == kPost) {
        const unsigned nw = grid_for(P.n_events * P.n_seg, fcsk::kBlock / fcsk::kWave);
        hipLaunchKernelGGL(fcsk::k_seg_count, dim3(P.n_seg_groups), dim3(fcsk::kBlock), 0, s, dP);
        hipLaunchKernelGGL(fcsk::k_seg_top, dim3(1), dim3(1024), 0, s, dP);
        hipLaunchKernelGGL(fcsk::k_seg_list, dim3(nw), dim3(fcsk::kBlock), 0, s, dP);
        // the emit pass is latency bound: 16 persistent workgroups per CU
        hipLaunchKernelGGL(fcsk::k_seg_emit, dim3(c->n_cu * 16), dim3(fcsk::kBlock), 0, s, dP);
    }
}

// instantiate (once per batch shape) and launch the graph of one part
int launch_graph(fcs_ctx* c, const Params& P, const GraphKey& key, int mode, int grid, int part)
{
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        enqueue_batch(c, P, mode, grid, part);
        HIPCHK(c, hipStreamEndCapture(c->stream, &g));
        const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(c, e);
        it = c->graphs.emplace(key, ge).first;
    }
    HIPCHK(c, hipGraphLaunch(it->second, c->stream));
    return FCS_OK;
}

int counters_error(fcs_ctx* c, const Counters& k)
{
    if (k.error & fcsk::kErrPdg) return fail(c, FCS_E_INVALID_ARG, "unknown particle pdg (use 11, 22, 211)");
    if (k.error & fcsk::kErrParticle)
        return fail(c, FCS_E_INVALID_ARG, "particle energy must be finite and > 0, eta/phi finite");
    if (k.error & fcsk::kErrOffsets) return fail(c, FCS_E_INVALID_ARG, "malformed event_offsets");
    if (k.error & fcsk::kErrOverride)
        return fail(c, FCS_E_INVALID_ARG,
                    "elayer_override holds a negative or non-finite energy, or one that gives a "
                    "(particle, layer) with hits a hit energy below FLT_MIN (x 2^26 with "
                    "hit_energy_fluct)");
    if (k.error & fcsk::kErrTooManyHits)
        return fail(c, FCS_E_CAPACITY, "more than 2^31-1 hits in one batch: split the batch");
    return FCS_OK;
}

// GPU time of a profiled synchronous launch sequence in its three parts:
// setup (and scans), the hit step (window pass and hit kernel, with the
// scans when the window pass runs beside them), compaction
struct PhaseMs {
    double setup = 0.0, hits = 0.0, compact = 0.0;
};

// the stream waits for the copy out of the staging set the call reuses
int wait_staged_copy(fcs_ctx* c)
{
    if (!c->post_wait) return FCS_OK;
    const hipEvent_t ev = c->post_wait;
    c->post_wait = nullptr;
    HIPCHK(c, hipStreamWaitEvent(c->stream, ev, 0));
    return FCS_OK;
}

// Run one launch sequence over a range of events and wait for it; with
// `async`, enqueue it followed by the fold of its counters into the
// context's running totals and return at once (*res is then zero).
int run_range(fcs_ctx* c, const fcs_sim_options* o, const Tuning& tu, const Shape& sh,
              const fcsk::Particle* d_particles, const long long* d_evoff, const float* d_override,
              float* dense_out, const fcs_sim_output* dout, bool want_hits, bool validate,
              bool use_graph, bool profile, Counters* res, PhaseMs* phase_ms, bool small_launch,
              bool async, bool per_task = false, char* scratch = nullptr)
{
    // a launch over few particles (per-event mode) gets a grid sized to its
    // tasks instead of filling the chip with idle persistent workgroups
    int grid = c->n_cu * tu.wg_per_cu;
    if (small_launch)
        grid = (int)std::min<long long>(grid, std::max<long long>(16, (sh.n_particles * c->n_layers + 3) / 4));
    std::memset(res, 0, sizeof *res);
    c->q_valid = false;
    // a batched call over device inputs leaves a work queue an adjoint call
    // may reuse
    // (not a no-allocation call: its queue lives in the shared scratch array)
    const bool keep = !small_launch && o->inputs_on_device && !o->placement_fp64 && !o->hit_energy_fluct &&
                      !scratch;
    for (int attempt = 0; attempt < 2; ++attempt) {
        char* blk = ring_take(c);
        if (!blk) return fail(c, FCS_E_HIP, "hipEventSynchronize on a parameter block failed");
        Params* P = (Params*)blk;
        Counters* hc = (Counters*)(blk + kCtrOffset);
        int rc = prepare(c, o, tu, sh, d_particles, d_evoff, d_override, dense_out, dout, want_hits,
                         async, P, scratch, !per_task);
        if (rc) return rc;
        const int mode = !dense_out ? kPrivate : (P->out_ids ? kDenseCompact : kDenseOnly);
        // asynchronous calls fold their totals into the context's running
        // totals: in the segment top pass, or in the last workgroup of the
        // count-reset pass of a dense-only call
        P->fold_acc = async ? (fcsk::AsyncAcc*)c->w_async.p : nullptr;
        P->validate = validate ? 1 : 0;
        std::memset(hc, 0, sizeof(Counters));
        HIPCHK(c, hipMemcpyAsync(c->cur_params, blk, kBlockBytes, hipMemcpyHostToDevice, c->stream));
        if ((rc = ring_sent(c))) return rc;
        GraphKey key{sh.n_particles, sh.n_events, mode, grid, kAll, P->placement_f64 + 2 * P->hit_fluct,
                     P->win_path};
        hipEvent_t k0 = c->ev_k0, k1 = c->ev_k1;
        if (profile && async) {
            // a free event pair for this call; the oldest pending one is read
            // first when all are in use
            if (c->prof_count == kProfRing) {
                const int old = c->prof_head;
                float ms = 0.f;
                HIPCHK(c, hipEventSynchronize(c->prof_ev[old][1]));
                HIPCHK(c, hipEventElapsedTime(&ms, c->prof_ev[old][0], c->prof_ev[old][1]));
                c->async_kernel_ms += ms;
                c->prof_head = (old + 1) % kProfRing;
                --c->prof_count;
            }
            const int slot = (c->prof_head + c->prof_count) % kProfRing;
            k0 = c->prof_ev[slot][0];
            k1 = c->prof_ev[slot][1];
            ++c->prof_count;
        }
        // a profiled synchronous call also times its setup and compaction
        const bool phases = profile && !async;
        if (phases) HIPCHK(c, hipEventRecord(c->ev_p0, c->stream));
        if (per_task) {
            // the per-(particle, layer) launch form: setup and scans, the
            // tasks' hit counts to the host, one launch per task with hits,
            // then the compaction
            enqueue_batch(c, *P, mode, grid, kPre);
            const long long nt = sh.n_particles * c->n_layers;
            c->h_task_n.resize((size_t)nt);
            HIPCHK(c, hipMemcpyAsync(c->h_task_n.data(), P->task_n, (size_t)nt * 4,
                                     hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            const Params* dP = (const Params*)c->cur_params;
            if (profile) HIPCHK(c, hipEventRecord(k0, c->stream));
            for (long long t = 0; t < nt; ++t) {
                if (c->h_task_n[(size_t)t] <= 0) continue;
                const dim3 g(grid_for(c->h_task_n[(size_t)t], fcsk::kBlock));
                if (P->placement_f64)
                    hipLaunchKernelGGL((fcsk::k_task_hits<true, false>), g, dim3(fcsk::kBlock),
                                       geo_lds_bytes(*P), c->stream, dP, (int)t);
                else if (P->hit_fluct)
                    hipLaunchKernelGGL((fcsk::k_task_hits<false, true>), g, dim3(fcsk::kBlock),
                                       geo_lds_bytes(*P), c->stream, dP, (int)t);
                else
                    hipLaunchKernelGGL((fcsk::k_task_hits<false, false>), g, dim3(fcsk::kBlock),
                                       geo_lds_bytes(*P), c->stream, dP, (int)t);
            }
            if (profile) HIPCHK(c, hipEventRecord(k1, c->stream));
            if ((rc = wait_staged_copy(c))) return rc;
            enqueue_batch(c, *P, mode, grid, kPost);
            if (phases) HIPCHK(c, hipEventRecord(c->ev_p1, c->stream));
            HIPCHK(c, hipGetLastError());
        } else if (use_graph && !profile && !(async && c->copy_deferred)) {
            if ((rc = wait_staged_copy(c))) return rc;
            if ((rc = launch_graph(c, *P, key, mode, grid, kAll))) return rc;
        } else {
            // profiled, or a copy to the host waits for the setup pass: the
            // hit kernels are launched on their own between the parts before
            // and after them (graphs)
            if (use_graph) {
                key.part = kPre;
                if ((rc = launch_graph(c, *P, key, mode, grid, kPre))) return rc;
            } else {
                enqueue_batch(c, *P, mode, grid, kPre);
            }
            // the previous batch's copy to the host starts beside this one's
            // window pass (the hit kernel leaves its workgroups no room)
            if (async && c->copy_deferred) {
                HIPCHK(c, hipEventRecord(c->ev_pre, c->stream));
                if ((rc = flush_host_copy(c, c->ev_pre))) return rc;
            }
            if (profile) HIPCHK(c, hipEventRecord(k0, c->stream));
            enqueue_batch(c, *P, mode, grid, kHits);
            if (profile) HIPCHK(c, hipEventRecord(k1, c->stream));
            // the staging set this batch compacts into is free once the
            // earlier copy out of it has ended
            if ((rc = wait_staged_copy(c))) return rc;
            if (use_graph) {
                key.part = kPost;
                if ((rc = launch_graph(c, *P, key, mode, grid, kPost))) return rc;
            } else {
                enqueue_batch(c, *P, mode, grid, kPost);
            }
            if (phases) HIPCHK(c, hipEventRecord(c->ev_p1, c->stream));
            HIPCHK(c, hipGetLastError());
        }
        if (async) {
            HIPCHK(c, hipGetLastError());
            if (keep && !P->win_path) {
                c->q_key = queue_key(o, tu, d_particles, d_evoff, sh.n_events, sh.n_particles, P->ev_base);
                c->q_params = *P;
                c->q_valid = true;
            }
            return FCS_OK;
        }
        HIPCHK(c, hipMemcpyAsync(hc, c->cur_params + kCtrOffset, sizeof(Counters),
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *res = *hc;
        if ((res->error & fcsk::kErrChunkCap) && scratch)
            return fail(c, FCS_E_INVALID_ARG,
                        "batch too large for fcs_simulate_events_noalloc: its work queue needs %d "
                        "entries, the scratch array holds %d (split the batch)", res->need_chunks,
                        P->chunk_cap);
        if ((res->error & fcsk::kErrChunkCap) && attempt == 0) {
            c->chunk_cap = (long long)res->need_chunks + 1024;
            continue;
        }
        if (profile && phase_ms) {
            float ms0 = 0.f, ms1 = 0.f, ms2 = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms0, c->ev_p0, k0));
            HIPCHK(c, hipEventElapsedTime(&ms1, k0, k1));
            HIPCHK(c, hipEventElapsedTime(&ms2, k1, c->ev_p1));
            phase_ms->setup += ms0;
            phase_ms->hits += ms1;
            phase_ms->compact += ms2;
        }
        const int rc2 = counters_error(c, *res);
        if (rc2 == FCS_OK && keep && !P->win_path) {
            c->q_key = queue_key(o, tu, d_particles, d_evoff, sh.n_events, sh.n_particles, P->ev_base);
            c->q_params = *P;
            c->q_valid = true;
        }
        return rc2;
    }
    return fail(c, FCS_E_HIP, "work queue sizing did not converge");
}


// host-side checks of host inputs
int check_host_inputs(fcs_ctx* c, const fcs_particle* parts, const int64_t* off, int64_t n_events)
{
    if (off[0] != 0) return fail(c, FCS_E_INVALID_ARG, "event_offsets[0] = %lld, must be 0", (long long)off[0]);
    for (int64_t e = 0; e < n_events; ++e)
        if (off[e + 1] < off[e])
            return fail(c, FCS_E_INVALID_ARG, "event_offsets decreases at event %lld", (long long)e);
    const int64_t N = off[n_events];
    for (int64_t i = 0; i < N; ++i) {
        const fcs_particle& p = parts[i];
        const int a = p.pdg < 0 ? -p.pdg : p.pdg;
        if (a != 11 && a != 22 && a != 211)
            return fail(c, FCS_E_INVALID_ARG, "particle %lld: unknown pdg %d (use 11, 22, 211)",
                        (long long)i, p.pdg);
        if (!finite_pos(p.e_mev))
            return fail(c, FCS_E_INVALID_ARG, "particle %lld: energy must be finite and > 0", (long long)i);
        if (!std::isfinite(p.eta) || !std::isfinite(p.phi) || std::fabs(p.phi) > 3.2f)
            return fail(c, FCS_E_INVALID_ARG, "particle %lld: eta/phi not finite or |phi| > 3.2",
                        (long long)i);
    }
    return FCS_OK;
}

// Common front half of simulate / query / backward: validate, bring inputs
// to the device, read the event offsets the host needs.
struct Inputs {
    const fcsk::Particle* d_particles = nullptr;
    const long long* d_evoff = nullptr;
    const float* d_override = nullptr;
    std::vector<int64_t> h_off;  // host copy of event_offsets
    long long N = 0;
    bool validate_on_device = false;
};

int stage_inputs(fcs_ctx* c, const fcs_particle* particles, const int64_t* event_offsets,
                 int64_t n_events, const fcs_sim_options* o, bool need_host_offsets, Inputs* in)
{
    if (!c->dry) {
        HIPCHK(c, hipSetDevice(c->device));
        int rc = activate_tables(c);  // tables of an asynchronous load, if any
        if (rc) return rc;
    }
    if (!c->has_geom || !c->has_param)
        return fail(c, FCS_E_NOT_LOADED, "load the geometry and the parametrization first");
    if (!o) return fail(c, FCS_E_INVALID_ARG, "options are NULL");
    if (n_events < 1) return fail(c, FCS_E_INVALID_ARG, "n_events = %lld, must be >= 1", (long long)n_events);
    if (!event_offsets) return fail(c, FCS_E_INVALID_ARG, "event_offsets is NULL");
    if (!(o->hit_energy_scale_mev > 0.f) || !std::isfinite(o->hit_energy_scale_mev))
        return fail(c, FCS_E_INVALID_ARG, "hit_energy_scale_mev must be finite and > 0");
    if (o->nhit_cap < 1) return fail(c, FCS_E_INVALID_ARG, "nhit_cap must be >= 1");
    if (!(o->min_layer_energy_mev > 0.0) || !std::isfinite(o->min_layer_energy_mev))
        return fail(c, FCS_E_INVALID_ARG, "min_layer_energy_mev must be finite and > 0");
    if (o->min_layer_energy_mev < min_hit_energy(o) * (double)o->nhit_cap)
        return fail(c, FCS_E_INVALID_ARG,
                    "min_layer_energy_mev = %g is below %g (FLT_MIN%s x nhit_cap): hit energies "
                    "could be subnormal", o->min_layer_energy_mev,
                    min_hit_energy(o) * (double)o->nhit_cap, o->hit_energy_fluct ? " x 2^26" : "");
    if (o->mode != FCS_MODE_BATCHED && o->mode != FCS_MODE_PER_EVENT && o->mode != FCS_MODE_PER_TASK)
        return fail(c, FCS_E_INVALID_ARG, "unknown mode %d", o->mode);
    if (o->placement_fp64 && o->hit_energy_fluct)
        return fail(c, FCS_E_INVALID_ARG, "placement_fp64 and hit_energy_fluct are exclusive");
    if (o->n_particles < 0) return fail(c, FCS_E_INVALID_ARG, "n_particles < 0");
    if (c->dry) {
        if (!o->inputs_on_device) {
            const long long N = event_offsets[n_events];
            if (N > 0 && !particles) return fail(c, FCS_E_INVALID_ARG, "particles is NULL");
            int rc = check_host_inputs(c, particles, event_offsets, n_events);
            if (rc) return rc;
        }
        return fail(c, FCS_E_NO_DEVICE, "context has no device (arguments are valid)");
    }
    HIPCHK(c, hipSetDevice(c->device));
    if (o->stream) {
        HIPCHK(c, hipEventRecord(c->ev_in, (hipStream_t)o->stream));
        HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_in, 0));
    }
    const int L = c->n_layers;
    if (!o->inputs_on_device) {
        in->N = event_offsets[n_events];
        if (in->N > 0 && !particles) return fail(c, FCS_E_INVALID_ARG, "particles is NULL");
        int rc = check_host_inputs(c, particles, event_offsets, n_events);
        if (rc) return rc;
        if (in->N >= (1LL << 25))
            return fail(c, FCS_E_INVALID_ARG, "%lld particles in one call, at most 2^25 - 1", in->N);
        if ((rc = upload(c, c->w_particles, (const fcsk::Particle*)particles, (size_t)in->N)) ||
            (rc = upload(c, c->w_evoff, (const long long*)event_offsets, (size_t)n_events + 1)))
            return rc;
        if (o->elayer_override) {
            for (long long i = 0; i < in->N * L; ++i)
                if (!std::isfinite(o->elayer_override[i]) || o->elayer_override[i] < 0.f)
                    return fail(c, FCS_E_INVALID_ARG, "elayer_override[%lld] negative or not finite", i);
            if ((rc = upload(c, c->w_override, o->elayer_override, (size_t)(in->N * L)))) return rc;
            in->d_override = (const float*)c->w_override.p;
        }
        in->d_particles = (const fcsk::Particle*)c->w_particles.p;
        in->d_evoff = (const long long*)c->w_evoff.p;
        if (need_host_offsets) in->h_off.assign(event_offsets, event_offsets + n_events + 1);
    } else {
        in->d_particles = (const fcsk::Particle*)particles;
        in->d_evoff = (const long long*)event_offsets;
        in->d_override = o->elayer_override;
        if (need_host_offsets) {
            in->h_off.resize((size_t)n_events + 1);
            HIPCHK(c, hipMemcpyAsync(in->h_off.data(), event_offsets, (n_events + 1) * sizeof(int64_t),
                                     hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            in->N = in->h_off[n_events];
            if (in->h_off[0] != 0)
                return fail(c, FCS_E_INVALID_ARG, "event_offsets[0] = %lld, must be 0", (long long)in->h_off[0]);
            for (int64_t e = 0; e < n_events; ++e)
                if (in->h_off[e + 1] < in->h_off[e])
                    return fail(c, FCS_E_INVALID_ARG, "event_offsets decreases at event %lld", (long long)e);
            if (o->n_particles > 0 && o->n_particles != in->N)
                return fail(c, FCS_E_INVALID_ARG, "n_particles = %lld but event_offsets[n_events] = %lld",
                            (long long)o->n_particles, in->N);
        } else if (o->n_particles > 0) {
            // checked against event_offsets[n_events] on the device
            in->N = o->n_particles;
        } else {
            int64_t last = 0;
            HIPCHK(c, hipMemcpyAsync(&last, event_offsets + n_events, sizeof(int64_t),
                                     hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            in->N = last;
        }
        if (in->N < 0 || in->N >= (1LL << 25))
            return fail(c, FCS_E_INVALID_ARG, "event_offsets[n_events] = %lld outside [0, 2^25)", in->N);
        if (in->N > 0 && !particles) return fail(c, FCS_E_INVALID_ARG, "particles is NULL");
        in->validate_on_device = true;
    }
    return FCS_OK;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// fcs_simulate_events, and with `noalloc` fcs_simulate_events_noalloc (the
// workspace carved from the device's scratch array; batched mode, device
// inputs and outputs, no captured graphs)
int simulate_impl(fcs_ctx* c, const fcs_particle* particles, const int64_t* event_offsets,
                  int64_t n_events, const fcs_sim_options* o, fcs_sim_output* out, bool noalloc)
{
    if (!c) return FCS_E_INVALID_ARG;
    if (!out) return fail(c, FCS_E_INVALID_ARG, "output struct is NULL");
    Tuning tu;
    int rc = o ? check_tuning(c, o, &tu) : fail(c, FCS_E_INVALID_ARG, "options are NULL");
    if (rc) return rc;
    if (noalloc && (o->mode != FCS_MODE_BATCHED || !o->inputs_on_device || !o->outputs_on_device))
        return fail(c, FCS_E_INVALID_ARG,
                    "fcs_simulate_events_noalloc needs batched mode and device inputs and outputs");
    const uint32_t f = o->outputs;
    if ((f & FCS_OUT_DENSE) && !out->cells) return fail(c, FCS_E_INVALID_ARG, "FCS_OUT_DENSE needs out->cells");
    if ((f & FCS_OUT_COMPACT) && (!out->cell_ids || !out->cell_e || !out->event_cell_offsets))
        return fail(c, FCS_E_INVALID_ARG, "FCS_OUT_COMPACT needs cell_ids, cell_e, event_cell_offsets");
    if ((f & FCS_OUT_COMPACT) && out->cell_capacity < 0)
        return fail(c, FCS_E_INVALID_ARG, "cell_capacity < 0");
    if ((f & FCS_OUT_HITS) && (!out->hit_eta || !out->hit_phi || !out->hit_e || !out->hit_cell ||
                               !out->task_hit_offsets || out->hit_capacity < 0))
        return fail(c, FCS_E_INVALID_ARG, "FCS_OUT_HITS needs hit_eta/phi/e/cell, task_hit_offsets, hit_capacity");
    if ((f & FCS_OUT_COUNTS) && !out->counts) return fail(c, FCS_E_INVALID_ARG, "FCS_OUT_COUNTS needs out->counts");
    if ((f & FCS_OUT_ELAYER) && !out->elayer) return fail(c, FCS_E_INVALID_ARG, "FCS_OUT_ELAYER needs out->elayer");
    const bool per_event = o->mode != FCS_MODE_BATCHED;  // per event, or per task within events
    const bool per_task = o->mode == FCS_MODE_PER_TASK;
    const bool async = o->async_launch != 0;
    // an asynchronous call may leave its compacted lists in pinned host
    // buffers (fcs_host_alloc): they are copied there beside the next batch
    const bool async_host = async && !o->outputs_on_device;
    if (async && (per_event || !o->inputs_on_device || o->n_particles <= 0 || (async_host && noalloc)))
        return fail(c, FCS_E_INVALID_ARG,
                    "async_launch needs batched mode, device inputs and n_particles (and device "
                    "outputs for fcs_simulate_events_noalloc)");
    if (async_host && f != FCS_OUT_COMPACT)
        return fail(c, FCS_E_INVALID_ARG, "async_launch with host outputs takes FCS_OUT_COMPACT alone");
    if (async_host && !c->dry &&
        (!pinned_host(out->cell_ids) || !pinned_host(out->cell_e) || !pinned_host(out->event_cell_offsets)))
        return fail(c, FCS_E_INVALID_ARG,
                    "async_launch with host outputs needs pinned cell_ids, cell_e and "
                    "event_cell_offsets (fcs_host_alloc)");
    // a deferred copy to the host waits for this call's setup pass only if
    // this call is one of the same kind
    if (!c->dry && !async_host && (rc = flush_host_copy(c))) return rc;
    Inputs in;
    if ((rc = stage_inputs(c, particles, event_offsets, n_events, o, per_event, &in))) return rc;
    char* const scratch = noalloc ? c->scratch : nullptr;
    if (noalloc && !scratch) return fail(c, FCS_E_NO_DEVICE, "context has no scratch array");
    const int L = c->n_layers;
    const long long N = in.N;
    const long long C = c->n_cells;

    // device-side output views (the caller's, or staging for host outputs)
    fcs_sim_output d = *out;
    const bool host_out = !o->outputs_on_device && !async_host;
    int hs = -1;  // staging set of an asynchronous call with host outputs
    if (async_host) {
        hs = c->hs_next;
        c->hs_next ^= 1;
        // the set is free once its last copy to the host has completed
        if (c->copy_deferred && c->dc.hs == hs && (rc = flush_host_copy(c))) return rc;
        if (c->copy_pending[hs]) {
            if (!per_event && in.N > 0) c->post_wait = c->ev_copied[hs];
            else HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_copied[hs], 0));
        }
        const size_t cap = (size_t)std::max<int64_t>(out->cell_capacity, 1);
        if (c->hs_ids[hs].bytes < cap * 8 || c->hs_e[hs].bytes < cap * 4 ||
            c->hs_off[hs].bytes < (size_t)(n_events + 1) * 8)
            HIPCHK(c, hipStreamSynchronize(c->copy_stream));  // a grown set frees the old one
        if ((rc = ensure(c, c->hs_ids[hs], cap * 8)) || (rc = ensure(c, c->hs_e[hs], cap * 4)) ||
            (rc = ensure(c, c->hs_off[hs], (size_t)(n_events + 1) * 8)))
            return rc;
        d.cell_ids = (int64_t*)c->hs_ids[hs].p;
        d.cell_e = (float*)c->hs_e[hs].p;
        d.event_cell_offsets = (int64_t*)c->hs_off[hs].p;
    }
    if (host_out) {
        if ((f & FCS_OUT_DENSE) && (rc = ensure(c, c->o_cells, (size_t)n_events * C * 4))) return rc;
        if (f & FCS_OUT_COMPACT) {
            if ((rc = ensure(c, c->o_ids, (size_t)std::max<int64_t>(out->cell_capacity, 1) * 8)) ||
                (rc = ensure(c, c->o_e, (size_t)std::max<int64_t>(out->cell_capacity, 1) * 4)) ||
                (rc = ensure(c, c->o_evoff, (size_t)(n_events + 1) * 8)))
                return rc;
            d.cell_ids = (int64_t*)c->o_ids.p;
            d.cell_e = (float*)c->o_e.p;
            d.event_cell_offsets = (int64_t*)c->o_evoff.p;
        }
        if (f & FCS_OUT_HITS) {
            const size_t hc = (size_t)std::max<int64_t>(out->hit_capacity, 1);
            if ((rc = ensure(c, c->o_heta, hc * 4)) || (rc = ensure(c, c->o_hphi, hc * 4)) ||
                (rc = ensure(c, c->o_he, hc * 4)) || (rc = ensure(c, c->o_hcell, hc * 4)) ||
                (rc = ensure(c, c->o_thoff, (size_t)(N * L + 1) * 8)))
                return rc;
            d.hit_eta = (float*)c->o_heta.p;
            d.hit_phi = (float*)c->o_hphi.p;
            d.hit_e = (float*)c->o_he.p;
            d.hit_cell = (int32_t*)c->o_hcell.p;
            d.task_hit_offsets = (int64_t*)c->o_thoff.p;
        }
        if ((f & FCS_OUT_COUNTS) && (rc = ensure(c, c->o_counts, (size_t)std::max<long long>(N * L, 1) * 4))) return rc;
        if ((f & FCS_OUT_ELAYER) && (rc = ensure(c, c->o_elayer, (size_t)std::max<long long>(N * L, 1) * 4))) return rc;
        d.cells = (f & FCS_OUT_DENSE) ? (float*)c->o_cells.p : nullptr;
        d.counts = (f & FCS_OUT_COUNTS) ? (int32_t*)c->o_counts.p : nullptr;
        d.elayer = (f & FCS_OUT_ELAYER) ? (float*)c->o_elayer.p : nullptr;
    }
    if (!(f & FCS_OUT_DENSE)) d.cells = nullptr;
    if (!(f & FCS_OUT_COMPACT)) {
        d.cell_ids = nullptr;
        d.cell_e = nullptr;
        d.event_cell_offsets = nullptr;
        d.cell_capacity = 0;
    }
    if (!(f & FCS_OUT_HITS)) {
        d.hit_eta = d.hit_phi = d.hit_e = nullptr;
        d.hit_cell = nullptr;
        d.task_hit_offsets = nullptr;
        d.hit_capacity = 0;
    }
    if (!(f & FCS_OUT_COUNTS)) d.counts = nullptr;
    if (!(f & FCS_OUT_ELAYER)) d.elayer = nullptr;
    const bool want_hits = (f & FCS_OUT_HITS) != 0;

    if (!async) HIPCHK(c, hipEventRecord(c->ev_start, c->stream));
    long long hits = 0, hits_out = 0, nnz = 0, items = 0;
    PhaseMs pm;
    const bool profile = o->profile != 0;
    if (N == 0) {
        // no particles: zero outputs only
        if (d.cells) HIPCHK(c, hipMemsetAsync(d.cells, 0, (size_t)n_events * C * 4, c->stream));
        if (d.event_cell_offsets)
            HIPCHK(c, hipMemsetAsync(d.event_cell_offsets, 0, (size_t)(n_events + 1) * 8, c->stream));
        if (d.task_hit_offsets) HIPCHK(c, hipMemsetAsync(d.task_hit_offsets, 0, 8, c->stream));
    } else if (!per_event) {
        Shape sh{N, 0, n_events, 0, 0, 0};
        Counters k;
        rc = run_range(c, o, tu, sh, in.d_particles, in.d_evoff, in.d_override, d.cells, &d,
                       want_hits, in.validate_on_device, o->use_graph != 0 && !scratch, profile, &k,
                       &pm, false, async, false, scratch);
        // a run that failed before its compaction still leaves the set's
        // copy ahead of whatever the stream does next
        if (int rcw = wait_staged_copy(c)) return rc ? rc : rcw;
        if (rc) return rc;
        hits = k.hits_total;
        hits_out = k.hits_out;
        nnz = k.nnz_total;
        items = (long long)k.n_chunks + k.n_tiles;
    } else {
        for (int64_t e = 0; e < n_events; ++e) {
            const long long p0 = in.h_off[e], p1 = in.h_off[e + 1];
            fcs_sim_output de = d;
            if (d.cells) de.cells = d.cells + e * C;
            if (d.counts) de.counts = d.counts + p0 * L;
            if (d.elayer) de.elayer = d.elayer + p0 * L;
            if (d.task_hit_offsets) de.task_hit_offsets = d.task_hit_offsets + p0 * L;
            if (d.event_cell_offsets) de.event_cell_offsets = d.event_cell_offsets + e;
            if (p1 == p0) {
                if (de.cells) HIPCHK(c, hipMemsetAsync(de.cells, 0, (size_t)C * 4, c->stream));
                if (de.event_cell_offsets) {
                    // an empty event: its offset is the running count
                    HIPCHK(c, hipMemcpyAsync(de.event_cell_offsets, &nnz, 8, hipMemcpyHostToDevice, c->stream));
                    HIPCHK(c, hipStreamSynchronize(c->stream));
                }
                continue;
            }
            Shape sh{p1 - p0, p0, 1, e, hits, nnz};
            const fcsk::Particle* dp = in.d_particles + p0;
            const float* dov = in.d_override ? in.d_override + p0 * L : nullptr;
            Counters k;
            rc = run_range(c, o, tu, sh, dp, in.d_evoff + e, dov, de.cells, &de, want_hits,
                           in.validate_on_device, false, profile, &k, &pm, true, false, per_task);
            if (rc) return rc;
            hits += k.hits_total;
            hits_out += k.hits_out;
            nnz += k.nnz_total;
            items += (long long)k.n_chunks + k.n_tiles;
        }
        if (d.event_cell_offsets)
            HIPCHK(c, hipMemcpyAsync(d.event_cell_offsets + n_events, &nnz, 8, hipMemcpyHostToDevice, c->stream));
        if (d.task_hit_offsets)
            HIPCHK(c, hipMemcpyAsync(d.task_hit_offsets + N * L, &hits, 8, hipMemcpyHostToDevice, c->stream));
    }
    if (async_host) {
        // the copy of this batch's lists to the host is enqueued by the next
        // call, to start after its setup pass: it then runs beside that
        // batch's window pass and hit kernel.  The setup pass's memory
        // accesses slow down the most under the host link's traffic, the
        // hit kernel's arithmetic the least; a copy kernel of a few
        // workgroups keeps that traffic low.  Any other entry point enqueues
        // it first.
        HIPCHK(c, hipEventRecord(c->ev_staged[hs], c->stream));
        if ((rc = flush_host_copy(c))) return rc;  // one the run above did not take
        fcs_ctx::HostCopy dc{};
        dc.hs = hs;
        dc.wgs = o->host_copy_workgroups > 0 ? o->host_copy_workgroups
                                             : (o->host_copy_workgroups == 0 ? kHostCopyWgs : 0);
        dc.n_events = n_events;
        dc.m = std::max<int64_t>(out->cell_capacity, 0);
        dc.h_ids = out->cell_ids;
        dc.h_e = out->cell_e;
        dc.h_off = out->event_cell_offsets;
        if (dc.wgs > 0) {  // the kernel stores through the device mapping
            void *h_ids = nullptr, *h_e = nullptr, *h_off = nullptr;
            HIPCHK(c, hipHostGetDevicePointer(&h_ids, out->cell_ids, 0));
            HIPCHK(c, hipHostGetDevicePointer(&h_e, out->cell_e, 0));
            HIPCHK(c, hipHostGetDevicePointer(&h_off, out->event_cell_offsets, 0));
            dc.h_ids = (int64_t*)h_ids;
            dc.h_e = (float*)h_e;
            dc.h_off = (int64_t*)h_off;
        }
        c->dc = dc;
        c->copy_deferred = true;
    }
    if (async) {
        // the caller's stream waits for the results; nothing is known yet
        HIPCHK(c, hipEventRecord(c->ev_done, c->stream));
        if (o->stream) HIPCHK(c, hipStreamWaitEvent((hipStream_t)o->stream, c->ev_done, 0));
        out->n_hits = out->n_hits_out_of_acceptance = -1;
        out->n_tasks = N * L;
        out->n_cells_nonzero = out->required_cell_capacity = out->required_hit_capacity = -1;
        out->n_work_items = -1;
        out->device_ms = out->kernel_ms = out->setup_ms = out->compact_ms = -1.0;
        return FCS_OK;
    }
    HIPCHK(c, hipEventRecord(c->ev_stop, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, c->ev_start, c->ev_stop);

    out->n_hits = hits;
    out->n_hits_out_of_acceptance = hits_out;
    out->n_tasks = N * L;
    out->n_cells_nonzero = nnz;
    out->required_cell_capacity = nnz;
    out->required_hit_capacity = hits;
    out->n_work_items = items;
    out->device_ms = ms;
    out->kernel_ms = pm.hits;
    out->setup_ms = pm.setup;
    out->compact_ms = pm.compact;

    if (host_out) {
        if (f & FCS_OUT_DENSE)
            HIPCHK(c, hipMemcpy(out->cells, d.cells, (size_t)n_events * C * 4, hipMemcpyDeviceToHost));
        if (f & FCS_OUT_COMPACT) {
            const size_t m = (size_t)std::min<long long>(nnz, out->cell_capacity);
            if (m) {
                HIPCHK(c, hipMemcpy(out->cell_ids, d.cell_ids, m * 8, hipMemcpyDeviceToHost));
                HIPCHK(c, hipMemcpy(out->cell_e, d.cell_e, m * 4, hipMemcpyDeviceToHost));
            }
            HIPCHK(c, hipMemcpy(out->event_cell_offsets, d.event_cell_offsets, (n_events + 1) * 8,
                                hipMemcpyDeviceToHost));
        }
        if (f & FCS_OUT_HITS) {
            const size_t m = (size_t)std::min<long long>(hits, out->hit_capacity);
            if (m) {
                HIPCHK(c, hipMemcpy(out->hit_eta, d.hit_eta, m * 4, hipMemcpyDeviceToHost));
                HIPCHK(c, hipMemcpy(out->hit_phi, d.hit_phi, m * 4, hipMemcpyDeviceToHost));
                HIPCHK(c, hipMemcpy(out->hit_e, d.hit_e, m * 4, hipMemcpyDeviceToHost));
                HIPCHK(c, hipMemcpy(out->hit_cell, d.hit_cell, m * 4, hipMemcpyDeviceToHost));
            }
            HIPCHK(c, hipMemcpy(out->task_hit_offsets, d.task_hit_offsets, (size_t)(N * L + 1) * 8,
                                hipMemcpyDeviceToHost));
        }
        if ((f & FCS_OUT_COUNTS) && N)
            HIPCHK(c, hipMemcpy(out->counts, d.counts, (size_t)(N * L) * 4, hipMemcpyDeviceToHost));
        if ((f & FCS_OUT_ELAYER) && N)
            HIPCHK(c, hipMemcpy(out->elayer, d.elayer, (size_t)(N * L) * 4, hipMemcpyDeviceToHost));
    }
    if ((f & FCS_OUT_COMPACT) && nnz > out->cell_capacity)
        return fail(c, FCS_E_CAPACITY, "cell_capacity %lld < %lld compacted cells",
                    (long long)out->cell_capacity, nnz);
    if ((f & FCS_OUT_HITS) && hits > out->hit_capacity)
        return fail(c, FCS_E_CAPACITY, "hit_capacity %lld < %lld hits", (long long)out->hit_capacity, hits);
    return FCS_OK;
}

}  // namespace

extern "C" {

int fcs_simulate_events(fcs_ctx* c, const fcs_particle* particles, const int64_t* event_offsets,
                        int64_t n_events, const fcs_sim_options* o, fcs_sim_output* out)
{
    const Range range("fcs_simulate_events");
    return simulate_impl(c, particles, event_offsets, n_events, o, out, false);
}

int fcs_simulate_events_noalloc(fcs_ctx* c, const fcs_particle* particles, const int64_t* event_offsets,
                                int64_t n_events, const fcs_sim_options* o, fcs_sim_output* out)
{
    const Range range("fcs_simulate_events_noalloc");
    return simulate_impl(c, particles, event_offsets, n_events, o, out, true);
}

int fcs_synchronize(fcs_ctx* c, fcs_async_stats* st)
{
    const Range range("fcs_synchronize");
    if (!c) return FCS_E_INVALID_ARG;
    if (st) std::memset(st, 0, sizeof *st);
    if (c->dry) return fail(c, FCS_E_NO_DEVICE, "context has no device");
    HIPCHK(c, hipSetDevice(c->device));
    int rc0 = flush_host_copy(c);
    if (rc0) return rc0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipStreamSynchronize(c->copy_stream));
    fcsk::AsyncAcc a;
    HIPCHK(c, hipMemcpy(&a, c->w_async.p, sizeof a, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemset(c->w_async.p, 0, sizeof a));
    double kms = c->async_kernel_ms;
    for (; c->prof_count > 0; --c->prof_count) {
        const int i = c->prof_head;
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->prof_ev[i][0], c->prof_ev[i][1]));
        kms += ms;
        c->prof_head = (i + 1) % kProfRing;
    }
    c->async_kernel_ms = 0.0;
    if (st) {
        st->n_calls = a.n_calls;
        st->n_hits = a.hits;
        st->n_hits_out_of_acceptance = a.hits_out;
        st->n_cells_nonzero = a.nnz;
        st->kernel_ms = kms;
    }
    Counters k{};
    k.error = a.error;
    int rc = counters_error(c, k);
    if (rc) return rc;
    if (a.error & fcsk::kErrCellCap)
        return fail(c, FCS_E_CAPACITY, "an asynchronous call had more compacted cells than cell_capacity");
    if (a.error & fcsk::kErrHitCap)
        return fail(c, FCS_E_CAPACITY, "an asynchronous call had more hits than hit_capacity");
    if (a.error & fcsk::kErrChunkCap)
        return fail(c, FCS_E_HIP, "an asynchronous call overflowed the chunk list");
    return FCS_OK;
}

int fcs_query_sizes(fcs_ctx* c, const fcs_particle* particles, const int64_t* event_offsets,
                    int64_t n_events, const fcs_sim_options* o, fcs_sizes* s)
{
    const Range range("fcs_query_sizes");
    if (!c) return FCS_E_INVALID_ARG;
    if (!s) return fail(c, FCS_E_INVALID_ARG, "sizes struct is NULL");
    Tuning tu;
    int rc = o ? check_tuning(c, o, &tu) : fail(c, FCS_E_INVALID_ARG, "options are NULL");
    if (rc) return rc;
    if (!c->dry && (rc = flush_host_copy(c))) return rc;
    Inputs in;
    if ((rc = stage_inputs(c, particles, event_offsets, n_events, o, false, &in))) return rc;
    std::memset(s, 0, sizeof *s);
    if (in.N == 0) return FCS_OK;
    char* blk = ring_take(c);
    if (!blk) return fail(c, FCS_E_HIP, "hipEventSynchronize on a parameter block failed");
    Params* P = (Params*)blk;
    Counters* hc = (Counters*)(blk + kCtrOffset);
    Shape sh{in.N, 0, n_events, 0, 0, 0};
    if ((rc = prepare(c, o, tu, sh, in.d_particles, in.d_evoff, nullptr, nullptr, nullptr, false,
                      false, P)))
        return rc;
    P->validate = in.validate_on_device ? 1 : 0;
    c->q_valid = false;  // the setup below overwrites the workspace's task arrays
    const Params* dP = (const Params*)c->w_params.p;
    std::memset(hc, 0, sizeof(Counters));
    HIPCHK(c, hipMemcpyAsync(c->w_params.p, blk, kBlockBytes, hipMemcpyHostToDevice, c->stream));
    if ((rc = ring_sent(c))) return rc;
    launch_setup(c->stream, dP, in.N, c->n_layers, c->n_cu);
    hipLaunchKernelGGL(fcsk::k_scan_group, dim3(P->n_scan_groups), dim3(fcsk::kScanThreads), 0, c->stream, dP);
    if (P->n_scan_groups > 1)
        hipLaunchKernelGGL(fcsk::k_scan_top, dim3(1), dim3(fcsk::kScanThreads), 0, c->stream, dP);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(hc, (char*)c->w_params.p + kCtrOffset, sizeof(Counters),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const Counters k = *hc;
    if ((rc = counters_error(c, k))) return rc;
    s->n_hits = k.hits_total;
    s->n_tasks = in.N * c->n_layers;
    s->max_cells = std::min<long long>(k.hits_total, (long long)n_events * c->n_cells);
    return FCS_OK;
}

int fcs_backward(fcs_ctx* c, const fcs_particle* particles, const int64_t* event_offsets,
                 int64_t n_events, const fcs_sim_options* o, const float* grad_cells,
                 float* grad_elayer, float* grad_weights)
{
    const Range range("fcs_backward");
    if (!c) return FCS_E_INVALID_ARG;
    if (!grad_cells) return fail(c, FCS_E_INVALID_ARG, "grad_cells is NULL");
    if ((uintptr_t)grad_weights & 15)
        return fail(c, FCS_E_INVALID_ARG, "grad_weights must be 16-byte aligned");
    Tuning tu;
    int rc = o ? check_tuning(c, o, &tu) : fail(c, FCS_E_INVALID_ARG, "options are NULL");
    if (rc) return rc;
    const bool async = o->async_launch != 0;
    if (async && (!o->inputs_on_device || o->n_particles <= 0))
        return fail(c, FCS_E_INVALID_ARG, "async_launch needs device inputs and n_particles");
    if (o->placement_fp64)
        return fail(c, FCS_E_INVALID_ARG, "placement_fp64 is a forward-only variant: the adjoint "
                                          "recomputes hits with the FP32 placement");
    if (!c->dry && (rc = flush_host_copy(c))) return rc;
    Inputs in;
    if ((rc = stage_inputs(c, particles, event_offsets, n_events, o, false, &in))) return rc;
    const long long nt = in.N * c->n_layers;
    // an asynchronous call returns once enqueued; the caller's stream waits
    // for its gradients, errors are reported by fcs_synchronize
    auto finish_async = [&]() -> int {
        HIPCHK(c, hipEventRecord(c->ev_done, c->stream));
        if (o->stream) HIPCHK(c, hipStreamWaitEvent((hipStream_t)o->stream, c->ev_done, 0));
        return FCS_OK;
    };
    if (in.N == 0) {
        if (grad_weights) HIPCHK(c, hipMemsetAsync(grad_weights, 0, (size_t)c->n_hist * 256 * 4, c->stream));
        if (async) return finish_async();
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return FCS_OK;
    }
    // The accumulators are zeroed when allocated; the passes that read them
    // (k_adj_elayer, k_adj_weights) clear what they read, so every call
    // finds them at zero.
    bool g_el = false, g_bins = false, g_mark = false;
    if ((rc = ensure(c, c->w_acc_el, (size_t)nt * 8, &g_el)) ||
        (rc = ensure(c, c->w_acc_bins, (size_t)c->n_hist * 256 * 8, &g_bins)) ||
        (rc = ensure(c, c->w_hist_mark, (size_t)c->n_hist, &g_mark)))
        return rc;
    if (g_el) HIPCHK(c, hipMemsetAsync(c->w_acc_el.p, 0, c->w_acc_el.bytes, c->stream));
    if (g_bins) HIPCHK(c, hipMemsetAsync(c->w_acc_bins.p, 0, c->w_acc_bins.bytes, c->stream));
    if (g_mark) HIPCHK(c, hipMemsetAsync(c->w_hist_mark.p, 0, c->w_hist_mark.bytes, c->stream));
    const Params* dP = (const Params*)c->w_params.p;
    hipStream_t s = c->stream;
    auto grads_to = [&](Params* P) {
        P->grad_cells = grad_cells;
        P->acc_elayer = (double*)c->w_acc_el.p;
        P->acc_bins = (double*)c->w_acc_bins.p;
        P->hist_mark = (uint8_t*)c->w_hist_mark.p;
        P->grad_elayer = grad_elayer;
        P->grad_weights = grad_weights;
    };
    // the adjoint passes; the last two run whatever gradients are asked for:
    // they also clear the accumulators
    auto launch_adjoint = [&](const Params& P) -> int {
        if (P.hit_fluct)
            hipLaunchKernelGGL((fcsk::k_adjoint<true>), dim3(c->n_cu * tu.wg_per_cu), dim3(fcsk::kBlock),
                               geo_lds_bytes(P), s, dP);
        else
            hipLaunchKernelGGL((fcsk::k_adjoint<false>), dim3(c->n_cu * tu.wg_per_cu), dim3(fcsk::kBlock),
                               geo_lds_bytes(P), s, dP);
        hipLaunchKernelGGL(fcsk::k_adj_elayer, dim3(grid_for(nt, 256)), dim3(256), 0, s, dP);
        hipLaunchKernelGGL(fcsk::k_adj_weights,
                           dim3(grid_for(std::min<long long>(c->n_hist, (long long)c->n_cu * 32),
                                         fcsk::kBlock / fcsk::kWave)),
                           dim3(fcsk::kBlock), 0, s, dP);
        HIPCHK(c, hipGetLastError());
        return FCS_OK;
    };
    const fcs_ctx::QueueKey key = queue_key(o, tu, in.d_particles, in.d_evoff, n_events, in.N,
                                            (long long)o->event_index_base);
    // The forward call's work queue, when asked for and still in the
    // workspace for these device inputs: only the adjoint passes run, on the
    // forward's parameter block; the forward's counters (the queue's sizes)
    // stay on the device and the queue's tickets are reset.
    if (o->reuse_forward_queue && o->inputs_on_device && c->q_valid && c->q_key == key) {
        char* blk = ring_take(c);
        if (!blk) return fail(c, FCS_E_HIP, "hipEventSynchronize on a parameter block failed");
        Params* P = (Params*)blk;
        Counters* hc = (Counters*)(blk + kCtrOffset);
        *P = c->q_params;
        P->validate = 0;
        // an asynchronous adjoint folds its error bits in k_adj_elayer (the
        // forward's, already folded, again: the fold is an OR)
        P->fold_acc = async ? (fcsk::AsyncAcc*)c->w_async.p : nullptr;
        grads_to(P);
        HIPCHK(c, hipMemcpyAsync(c->w_params.p, blk, sizeof(Params), hipMemcpyHostToDevice, s));
        if ((rc = ring_sent(c))) return rc;
        hipLaunchKernelGGL(fcsk::k_fill_u32, dim3(1), dim3(256), 0, s, (uint32_t*)c->w_queue.p,
                           (long long)fcsk::kQueueInts, 0u);
        if ((rc = launch_adjoint(*P))) return rc;
        if (async) return finish_async();
        HIPCHK(c, hipMemcpyAsync(hc, (char*)c->w_params.p + kCtrOffset, sizeof(Counters),
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        const Counters k = *hc;
        if (!(k.error & fcsk::kErrChunkCap)) return counters_error(c, k);
        // the forward's chunk list had overflowed: rebuild below
    }
    c->q_valid = false;  // the setup below rebuilds the workspace
    for (int attempt = 0; attempt < 2; ++attempt) {
        char* blk = ring_take(c);
        if (!blk) return fail(c, FCS_E_HIP, "hipEventSynchronize on a parameter block failed");
        Params* P = (Params*)blk;
        Counters* hc = (Counters*)(blk + kCtrOffset);
        Shape sh{in.N, 0, n_events, 0, 0, 0};
        if ((rc = prepare(c, o, tu, sh, in.d_particles, in.d_evoff, in.d_override, nullptr, nullptr,
                          false, async, P)))
            return rc;
        P->validate = in.validate_on_device ? 1 : 0;
        // an asynchronous adjoint folds its error bits in k_adj_elayer
        P->fold_acc = async ? (fcsk::AsyncAcc*)c->w_async.p : nullptr;
        grads_to(P);
        std::memset(hc, 0, sizeof(Counters));
        HIPCHK(c, hipMemcpyAsync(c->w_params.p, blk, kBlockBytes, hipMemcpyHostToDevice, s));
        if ((rc = ring_sent(c))) return rc;
        launch_setup(s, dP, in.N, c->n_layers, c->n_cu);
        hipLaunchKernelGGL(fcsk::k_scan_group, dim3(P->n_scan_groups), dim3(fcsk::kScanThreads), 0, s, dP);
        if (P->n_scan_groups > 1)
            hipLaunchKernelGGL(fcsk::k_scan_top, dim3(1), dim3(fcsk::kScanThreads), 0, s, dP);
        hipLaunchKernelGGL(fcsk::k_scan_write, dim3(P->n_scan_blocks), dim3(fcsk::kBlock), 0, s, dP);
        if ((rc = launch_adjoint(*P))) return rc;
        if (async) return finish_async();
        HIPCHK(c, hipMemcpyAsync(hc, (char*)c->w_params.p + kCtrOffset, sizeof(Counters),
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        const Counters k = *hc;
        if ((k.error & fcsk::kErrChunkCap) && attempt == 0) {
            c->chunk_cap = (long long)k.need_chunks + 1024;
            continue;
        }
        return counters_error(c, k);
    }
    return fail(c, FCS_E_HIP, "work queue sizing did not converge");
}

}  // extern "C"
