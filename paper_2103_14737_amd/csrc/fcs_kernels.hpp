// Kernels of the batched hit simulation on gfx950 (wave64).
//
// Pipeline of one batch (all launches read one device-resident Params block,
// so the sequence can be captured once in a hipGraph and replayed):
//   k_setup        per (particle, layer): parametrization set, Dirichlet layer
//                  energy, Poisson hit count, Ehit (Listing 1); per-block
//                  sums for the task scan
//   k_scan_group / k_scan_top / k_scan_write
//                  scans of the task hit counts -> work queue: chunks of
//                  large tasks, packed tiles of small tasks
//   k_windows      batches of many-particle events: the small tasks by cell
//                  window, summed in LDS and added with coalesced atomics
//                  (on a second stream beside the scans when it writes no
//                  hit lists)
//   k_hits         persistent: pulls work items from a ticket counter; per
//                  hit Philox draw, inverse-CDF bin, placement, cell lookup,
//                  deposit (sim_a of the CUDA Implementation section)
//   k_seg_count / k_seg_top / k_seg_list / k_seg_emit
//                  ordered gather of the hit cells as (cell_id, E) and
//                  sparse reset of the accumulator (sim_ct and clean);
//                  k_flags_reset instead for calls with a dense output only
#pragma once

#include "fcs_math.hpp"

namespace fcsk {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kBins = 256;
constexpr int kGuide = 1024;       // guide entries per histogram (top 10 bits of u0)
constexpr int kChunkMax = 32768;   // hits per chunk (per-cell counts are 16-bit)
constexpr int kHashProbes = 16;
constexpr uint32_t kEmpty = 0xffffffffu;
constexpr int kSegPerWave = 8;            // segments counted by one wave
constexpr int kTileMax = 512;             // max hits of one packed tile (one wave)
constexpr int kQueues = 8;                // work-queue ranges (one ticket each)
constexpr int kQueueStride = 64;          // ints between tickets: one 256-byte line each
// the queue block: kQueues tickets, kQueues drained flags, then the ticket of
// the window pass (k_windows)
constexpr int kWinTicket = 2 * kQueues;
constexpr int kQueueInts = (2 * kQueues + 1) * kQueueStride;

struct Particle {
    int32_t pdg;
    float e;
    float eta;
    float phi;
};

// device counters of one launch sequence
struct Counters {
    long long hits_total;
    long long hits_out;
    long long nnz_total;
    int32_t n_chunks;
    int32_t n_small_hits;
    int32_t n_small_tasks;
    int32_t n_tiles;
    int32_t error;        // bit set, see kErr*
    int32_t need_chunks;  // chunk entries required when over capacity
    uint32_t done;        // workgroups of the count-reset pass that finished
    int32_t max_event_particles;  // window pass: particles of the largest event
    long long n_blk_list; // nonzero 64-cell blocks listed by the compaction
};

// running totals of the asynchronous calls of a context (device memory)
struct AsyncAcc {
    long long n_calls;
    long long hits;
    long long hits_out;
    long long nnz;
    int32_t error;  // union of the calls' error bits
    int32_t pad;
};

enum : int32_t {
    kErrPdg = 1,          // unknown particle type
    kErrParticle = 2,     // non-finite / non-positive inputs
    kErrOffsets = 4,      // malformed event offsets
    kErrTooManyHits = 8,  // more than 2^31-1 hits in one batch
    kErrChunkCap = 16,    // chunk list capacity exceeded (internal retry)
    kErrOverride = 32,    // negative or non-finite override, or a subnormal hit energy from it
    kErrCellCap = 64,     // compacted cells beyond the output capacity (async calls)
    kErrHitCap = 128,     // hits beyond the hit-list capacity (async calls)
};

struct Params {
    // geometry
    long long n_cells;
    int32_t n_layers, n_regions;
    int32_t n_blk;     // flag stride per event in 64-cell blocks (a power of two)
    int32_t blk_shift; // log2(n_blk)
    int32_t n_seg;     // compaction segments (kSegBlocks flag blocks) per event
    const float* reg_eta_lo;
    const float* reg_eta_hi;
    const float* reg_inv_deta;
    const float* reg_inv_dphi;
    const float* reg_phi_lo;
    const int32_t* reg_neta;
    const int32_t* reg_nphi;
    const int32_t* reg_offset;
    const float* layer_inv_r;
    const long long* cell_id;
    // parametrization
    int32_t n_types, n_ebins, n_etabins;
    float r_max;
    const float* e_edges;
    const float* eta_edges;
    const float* alpha;
    const float* cum;
    const uint8_t* guide;
    const float* weights;
    // this call
    uint32_t key0, key1;
    unsigned long long ev_base;
    long long n_particles;   // particles of this launch
    long long part_base;     // index of its first particle in the caller's arrays
    long long n_events;
    long long n_tasks;
    const Particle* particles;
    const long long* ev_off;
    const float* elayer_override;
    float scale;
    int32_t cap;
    double min_e;
    float ehit_min;          // smallest positive hit energy an override may give
    int32_t chunk_hits, big_thr, tile_hits;
    int32_t want_hits;
    int32_t clean_cells;  // reset the accumulator while compacting
    int32_t chunk_cap;
    int32_t n_scan_blocks;
    int32_t n_scan_groups;
    int32_t setup_sub;     // scan blocks per setup workgroup
    int32_t placement_f64; // hit kernels place hits in FP64 (chain variant)
    int32_t hit_fluct;     // per-hit energy fluctuation (chain variant)
    int32_t validate;      // check device-resident inputs in the setup
    int32_t n_seg_groups;  // groups of kSegGroup segments
    // window pass (multi-particle events): the small tasks of each (event,
    // cell window of a layer, range of win_parts particles) are deposited by
    // k_windows instead of the tiles of k_hits
    int32_t win_path;
    int32_t win_parts;     // particles per work item of the window pass
    int32_t n_windows;
    const int4* geo_windows;  // [n_windows * 2] see WinRec
    unsigned long long* task_nT;  // window pass: hits | Ehit bits << 32 of task (p, l) at l * n_particles + p
    // workspace
    int32_t* task_n;
    float* task_ehit;
    int32_t* part_ev;
    uint32_t* part_p;
    int32_t* part_set;
    int32_t* blk_sums;   // [n_scan_blocks * 4]
    int32_t* blk_offs;   // [n_scan_blocks * 4] prefixes within the block's scan group
    long long* grp_hits; // [n_scan_groups] hits of each scan group
    int32_t* grp_rest;   // [n_scan_groups * 4] (-, chunks, small hits, small tasks) of each group
    int32_t* grp_offs;   // [n_scan_groups * 4] exclusive prefixes of the groups
    int32_t* task_hoff;  // [n_tasks] when want_hits
    int4* chunks;        // [chunk_cap] (task key, first hit, count, -)
    int4* small_rec;     // [2 * n_tasks] records of the small tasks
    const int4* geo_layers;   // [n_layers * 3] per-layer lookup records
    const int4* geo_regions;  // [n_layers * n_regions * 2] per-region records
    int32_t* tile_first; // [n_tasks + 1]
    float* cells;        // [n_events * n_cells] accumulator
    uint8_t* flags;      // [n_events * n_blk]
    long long* seg_off;  // [n_events * n_seg] (nonzero blocks << 32 | nonzero cells) before the
                         // segment, within its group of kSegGroup
    long long* seg_blk;  // [n_seg_groups] group totals, then their exclusive prefixes
    unsigned long long* blk_list;  // [n_events * n_seg * kSegBlocks] position << 32 | (event << blk_shift | block)
    Counters* ctr;
    AsyncAcc* fold_acc;   // asynchronous calls with compaction: k_seg_top folds the totals here
    int32_t* queue;      // [kQueueInts]: tickets, drained flags, window-pass ticket
    // outputs (device)
    float* out_elayer;
    int32_t* out_counts;
    long long* out_ids;
    float* out_e;
    long long out_cap;
    long long* out_ev_off;
    float* hit_eta;
    float* hit_phi;
    float* hit_e;
    int32_t* hit_cell;
    long long hit_cap;
    long long hit_base;      // hit-list position of this launch's first hit
    long long out_base;      // compacted position of this launch's first cell
    long long* out_task_hoff;
    // adjoint
    const float* grad_cells;
    double* acc_elayer;   // [n_tasks] FP64 sums of g over in-acceptance hits
    double* acc_bins;     // [n_hist * 256] FP64 sums of g * Ehit
    uint8_t* hist_mark;   // [n_hist] 1 where acc_bins may hold sums (set by the adjoint)
    float* grad_elayer;
    float* grad_weights;
    long long n_hist;
};

// ------------------------------------------------------------ utilities ---
// Pointers read from the Params block are generic; G() retypes them into the
// global address space so that accesses compile to global (not flat) memory
// instructions.  Atomics on such pointers go through the helpers below.
#define FCS_AS_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ FCS_AS_GLOBAL T* G(T* p)
{
    return (FCS_AS_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ const FCS_AS_GLOBAL T* G(const T* p)
{
    return (const FCS_AS_GLOBAL T*)p;
}

// relaxed device-scope atomics on global memory; the FP adds use the native
// instructions (denormal inputs are outside the value ranges used here)
__device__ __forceinline__ void gadd(FCS_AS_GLOBAL float* p, float v)
{
    [[clang::atomic(ignore_denormal_mode)]] {
        (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}
__device__ __forceinline__ void gadd(FCS_AS_GLOBAL double* p, double v)
{
    [[clang::atomic(ignore_denormal_mode)]] {
        (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}
// 16-byte records (particles, work items, scan partials) move as native int
// vectors, which load and store from the global address space directly
typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

__device__ __forceinline__ Particle load_particle(const Particle* base, long long i)
{
    const v4i v = ((const FCS_AS_GLOBAL v4i*)base)[i];
    Particle p;
    p.pdg = v.x;
    p.e = __int_as_float(v.y);
    p.eta = __int_as_float(v.z);
    p.phi = __int_as_float(v.w);
    return p;
}
__device__ __forceinline__ int4 load_i4(const int4* base, long long i)
{
    const v4i v = ((const FCS_AS_GLOBAL v4i*)base)[i];
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void store_i4(int4* base, long long i, int4 x)
{
    v4i v;
    v.x = x.x;
    v.y = x.y;
    v.z = x.z;
    v.w = x.w;
    ((FCS_AS_GLOBAL v4i*)base)[i] = v;
}

template <typename T>
__device__ __forceinline__ T gfetch_add(FCS_AS_GLOBAL T* p, T v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void gor(FCS_AS_GLOBAL T* p, T v)
{
    (void)__hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void gmax(FCS_AS_GLOBAL T* p, T v)
{
    (void)__hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// the window pass needs the particle count of the largest event: the first
// particle of each event reports its event's count
__device__ __forceinline__ void note_event_size(const Params& P, int ev, uint32_t pin)
{
    if (P.win_path && pin == 0)
        gmax(&G(P.ctr)->max_event_particles, (int32_t)(G(P.ev_off)[ev + 1] - G(P.ev_off)[ev]));
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const T t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

// inclusive scan (sum, or max of values >= 0) over a wave with DPP moves:
// shifts by 1, 2, 4 and 8 lanes within each row of 16 (lanes shifted in from
// outside the row read 0), then the last lane of rows 0 and 2 into rows 1 and
// 3, then lane 31 into rows 2 and 3.  No LDS round trips, unlike __shfl_up.
template <bool kMax>
__device__ __forceinline__ int wave_scan_dpp(int v)
{
#define FCS_DPP_STEP(ctrl, rows)                                              \
    {                                                                          \
        const int t = __builtin_amdgcn_update_dpp(0, v, ctrl, rows, 0xf, false); \
        v = kMax ? (t > v ? t : v) : v + t;                                    \
    }
    FCS_DPP_STEP(0x111, 0xf)  // row_shr:1
    FCS_DPP_STEP(0x112, 0xf)  // row_shr:2
    FCS_DPP_STEP(0x114, 0xf)  // row_shr:4
    FCS_DPP_STEP(0x118, 0xf)  // row_shr:8
    FCS_DPP_STEP(0x142, 0xa)  // row_bcast:15 into rows 1 and 3
    FCS_DPP_STEP(0x143, 0xc)  // row_bcast:31 into rows 2 and 3
#undef FCS_DPP_STEP
    return v;
}

__device__ __forceinline__ int4 add4(int4 a, int4 b) { return make_int4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
__device__ __forceinline__ int4 sub4(int4 a, int4 b) { return make_int4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w); }

__device__ __forceinline__ int4 wave_incl_scan4(int4 v)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int4 t;
        t.x = __shfl_up(v.x, d, kWave);
        t.y = __shfl_up(v.y, d, kWave);
        t.z = __shfl_up(v.z, d, kWave);
        t.w = __shfl_up(v.w, d, kWave);
        if (lane >= d) v = add4(v, t);
    }
    return v;
}

// exclusive block scan of int4 over 256 threads; also returns the total
__device__ __forceinline__ int4 block_excl_scan4(int4 v, int4& total)
{
    __shared__ int4 wsum[kBlock / kWave];
    const int wave = threadIdx.x / kWave;
    const int4 inc = wave_incl_scan4(v);
    if (lane_id() == kWave - 1) wsum[wave] = inc;
    __syncthreads();
    int4 off = make_int4(0, 0, 0, 0), tot = make_int4(0, 0, 0, 0);
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        const int4 s = wsum[w];
        if (w < wave) off = add4(off, s);
        tot = add4(tot, s);
    }
    __syncthreads();
    total = tot;
    return add4(sub4(inc, v), off);
}


// sum over a workgroup of kThreads threads (every thread calls it)
template <int kThreads = kBlock>
__device__ __forceinline__ long long block_sum_ll(long long v)
{
    __shared__ long long red[kThreads / kWave];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    if (lane_id() == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    long long t = 0;
#pragma unroll
    for (int w = 0; w < kThreads / kWave; ++w) t += red[w];
    __syncthreads();
    return t;
}


// ---------------------------------------------------- set selection (a1) ---
__device__ __forceinline__ int select_set(const Params& P, int pdg, float e, float eta)
{
    const int apdg = pdg < 0 ? -pdg : pdg;
    const int t = apdg == 11 ? 0 : apdg == 22 ? 1 : apdg == 211 ? 2 : -1;
    if (t < 0) return -1;
    int ie = 0;
    for (int k = 1; k < P.n_ebins; ++k) ie += (e >= G(P.e_edges)[k]) ? 1 : 0;
    const float ae = fabsf(eta);
    int ih = 0;
    for (int k = 1; k < P.n_etabins; ++k) ih += (ae >= G(P.eta_edges)[k]) ? 1 : 0;
    return (t * P.n_ebins + ie) * P.n_etabins + ih;
}

// largest e with ev_off[e] <= gp
template <typename Ptr>
__device__ __forceinline__ int find_event(Ptr ev_off, long long n_events, long long gp)
{
    long long lo = 0, hi = n_events - 1;
    while (lo < hi) {
        const long long mid = (lo + hi + 1) >> 1;
        if (ev_off[mid] <= gp) lo = mid;
        else hi = mid - 1;
    }
    return (int)lo;
}

// ------------------------------------------------------------- fills ---
__global__ void k_fill_u32(uint32_t* __restrict__ p, long long n, uint32_t v)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// Copy of an asynchronous call's compacted lists to pinned host memory by a
// few workgroups of the copy stream: the event offsets, then of each list
// the entries the batch wrote (the total in offsets[n_events], at most
// `cap`).  The stores cross the host link; with few waves in flight the
// kernels beside them keep the rest of the chip.  16-byte moves where the
// source and destination are both 16-byte aligned (eight loads in flight per
// thread before their stores: a workgroup's rate is set by how many bytes it
// has in flight; loads and stores marked streaming, so that the lists do not
// displace the tables the batch beside them reads from L2), element moves
// otherwise.
template <typename T>
__device__ void copy_to_host(const T* __restrict__ src, T* __restrict__ dst, long long n, long long gid,
                             long long stride)
{
    constexpr long long kPer = 16 / sizeof(T);
    constexpr int kUnroll = 8;
    if ((((uintptr_t)src | (uintptr_t)dst) & 15) == 0) {
        const long long nv = n / kPer;
        const v4i* s4 = reinterpret_cast<const v4i*>(src);
        v4i* d4 = reinterpret_cast<v4i*>(dst);
        long long i = gid;
        for (; i + (kUnroll - 1) * stride < nv; i += kUnroll * stride) {
            v4i v[kUnroll];
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) v[k] = __builtin_nontemporal_load(s4 + i + k * stride);
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) __builtin_nontemporal_store(v[k], d4 + i + k * stride);
        }
        for (; i < nv; i += stride) __builtin_nontemporal_store(s4[i], d4 + i);
        for (long long i = nv * kPer + gid; i < n; i += stride) dst[i] = src[i];
    } else {
        for (long long i = gid; i < n; i += stride) dst[i] = src[i];
    }
}

__global__ __launch_bounds__(kBlock) void k_copy_out(const int64_t* __restrict__ ids, const float* __restrict__ e,
                                                     const int64_t* __restrict__ off, int64_t* h_ids, float* h_e,
                                                     int64_t* h_off, long long n_events, long long cap)
{
    const long long gid = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long stride = (long long)gridDim.x * kBlock;
    const long long m = min(max(off[n_events], 0LL), cap);
    copy_to_host(off, h_off, n_events + 1, gid, stride);
    copy_to_host(ids, h_ids, m, gid, stride);
    copy_to_host(e, h_e, m, gid, stride);
}

__global__ void k_fill_u8(uint8_t* __restrict__ p, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

// zero the caller's dense cell buffer of this launch (read from Params so a
// captured graph can be replayed on other buffers)
__global__ void k_fill_dense(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const long long n = P.n_events * P.n_cells;
    auto p = G(P.cells);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// ---------------------------------------------- parametrization tables ---
// cumulative FP32 table per histogram: FP64 running sum over the FP64 total,
// last entry forced to 1.  A workgroup of 64 threads takes 64 histograms:
// their weights are loaded into LDS with coalesced reads (rows padded to 257
// words, so that the threads' row walks fall into distinct banks), each
// thread sums its own histogram left to right, and the tables are stored
// back coalesced.
constexpr int kCumHist = 64;
constexpr int kCumPad = kBins + 1;
__global__ __launch_bounds__(kCumHist) void k_build_cum(const float* __restrict__ w, float* __restrict__ cum,
                                                        long long n_hist)
{
    __shared__ float s_w[kCumHist * kCumPad];
    const long long h0 = (long long)blockIdx.x * kCumHist;
    const int nh = (int)min((long long)kCumHist, n_hist - h0);
    for (int i = threadIdx.x; i < nh * kBins; i += kCumHist)
        s_w[(i / kBins) * kCumPad + (i % kBins)] = w[h0 * kBins + i];
    __syncthreads();
    if ((int)threadIdx.x < nh) {
        float* row = s_w + threadIdx.x * kCumPad;
        double tot = 0.0;
        for (int b = 0; b < kBins; ++b) tot = tot + (double)row[b];
        double acc = 0.0;
        for (int b = 0; b < kBins; ++b) {
            acc = acc + (double)row[b];
            row[b] = (float)(acc / tot);
        }
        row[kBins - 1] = 1.0f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nh * kBins; i += kCumHist)
        cum[h0 * kBins + i] = s_w[(i / kBins) * kCumPad + (i % kBins)];
}

// guide table: g[j] = first bin with cum > j / kGuide, so that a u0 in
// [j, j+1) / kGuide has its bin in [g[j], g[j+1]] (the last entry's upper
// end is the last bin).  j / kGuide is exact in FP32 and cum is
// nondecreasing with cum[last] = 1, so bin b is g[j] exactly for
// ceil(kGuide cum[b-1]) <= j < ceil(kGuide cum[b]) (cum[-1] = 0): one wave
// per histogram, four bins per lane, each writing its run of entries.
__global__ __launch_bounds__(kBlock) void k_build_guide(const float* __restrict__ cum,
                                                        uint8_t* __restrict__ guide, long long n_hist)
{
    const long long h = (long long)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (h >= n_hist) return;
    const int lane = lane_id();
    const float* c = cum + h * kBins;
    uint8_t* g = guide + h * kGuide;
#pragma unroll
    for (int k = 0; k < kBins / kWave; ++k) {
        const int b = lane * (kBins / kWave) + k;
        const float lo = b ? c[b - 1] : 0.0f;
        const int j0 = (int)ceilf(lo * (float)kGuide);
        const int j1 = min((int)ceilf(c[b] * (float)kGuide), kGuide);
        for (int j = j0; j < j1; ++j) g[j] = (uint8_t)b;
    }
}

// Input checks of device-resident inputs, made by the setup kernels: each
// particle by the thread that loads it, the offsets grid-stride.  A failed
// check sets an error bit that the call reports; the batch still runs (every
// index stays in range: events come from a clamped search, hit counts are
// capped) and its outputs are unspecified.
__device__ __forceinline__ int particle_errors(const Particle& pt)
{
    int err = 0;
    const int a = pt.pdg < 0 ? -pt.pdg : pt.pdg;
    if (a != 11 && a != 22 && a != 211) err |= kErrPdg;
    if (!(pt.e > 0.0f) || !isfinite(pt.e) || !isfinite(pt.eta) || !isfinite(pt.phi) || fabsf(pt.phi) > 3.2f)
        err |= kErrParticle;
    return err;
}

__device__ __forceinline__ void check_offsets(const Params& P)
{
    const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    int err = 0;
    for (long long i = i0; i < P.n_events; i += stride)
        if (G(P.ev_off)[i] > G(P.ev_off)[i + 1]) err |= kErrOffsets;
    if (i0 == 0 &&
        (G(P.ev_off)[0] != P.part_base || G(P.ev_off)[P.n_events] != P.part_base + P.n_particles))
        err |= kErrOffsets;
    if (err) gor(&G(P.ctr)->error, err);
}

// ------------------------------------------- per-task setup (a1 - a3) ---
// Per (particle, layer) task: the Gamma draw, the Dirichlet normalization
// over the particle's layers (in LDS), the Poisson hit count and Ehit.
//
// (hits, chunks, small hits, small tasks) of a task with n hits
__device__ __forceinline__ int4 task_terms(const Params& P, int n)
{
    const bool big = n >= P.big_thr;
    return make_int4(n, big ? (n + P.chunk_hits - 1) / P.chunk_hits : 0, (!big && n > 0) ? n : 0,
                     (!big && n > 0) ? 1 : 0);
}

// Batches too small to give every CU several workgroups of several scan
// blocks: one thread per task, one scan block (kBlock / L particles) per
// workgroup.
// a task's (hits, Ehit) pair as the window pass reads it
__device__ __forceinline__ unsigned long long task_pair(int n, float ehit)
{
    return (unsigned long long)(uint32_t)n | ((unsigned long long)__float_as_uint(ehit) << 32);
}

__global__ __launch_bounds__(kBlock) void k_setup_one(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    __shared__ double g_s[kBlock];
    __shared__ double s_mu[kBlock];
    __shared__ uint32_t s_pin[kBlock], s_evg[kBlock];
    __shared__ int s_n[kBlock];
    __shared__ uint16_t s_list[kBlock];
    __shared__ int s_cnt[2];
    const int L = P.n_layers;
    const int ppb = kBlock / L;
    const int tid = threadIdx.x;
    const int lp = tid / L;
    const int l = tid - lp * L;
    const long long gp = (long long)blockIdx.x * ppb + lp;
    const bool active = lp < ppb && gp < P.n_particles;
    if (P.validate) check_offsets(P);
    if (blockIdx.x == 0 && tid == 0) G(P.queue)[kWinTicket * kQueueStride] = 0;  // the window pass's ticket
    Particle pt = {0, 0.f, 0.f, 0.f};
    int set = -1, ev = 0;
    uint32_t pin = 0, evg = 0;
    double g = 0.0;
    if (active) {
        pt = load_particle(P.particles, gp);
        if (P.validate && l == 0) {
            const int err = particle_errors(pt);
            if (err) gor(&G(P.ctr)->error, err);
        }
        ev = find_event(G(P.ev_off), P.n_events, P.part_base + gp);
        pin = (uint32_t)(P.part_base + gp - G(P.ev_off)[ev]);
        evg = (uint32_t)(P.ev_base + (unsigned long long)ev);
        if (l == 0) note_event_size(P, ev, pin);
        set = select_set(P, pt.pdg, pt.e, pt.eta);
        if (set >= 0) {
            const int ty = set / (P.n_ebins * P.n_etabins);
            const double alpha = (double)G(P.alpha)[ty * L + l];
            const double a = alpha < 1.0 ? alpha + 1.0 : alpha;
            const double d = a - 1.0 / 3.0;
            const double c = 1.0 / sqrt(9.0 * d);
            uint32_t j = 0, w = 0;
            while (!gamma_try<0>(d, c, j, P.key0, P.key1, (uint32_t)l, pin, evg, &g, &w) && ++j < 64) {
            }
            g = j < 64 ? gamma_boost<0>(g, alpha, w) : d;
        }
    }
    g_s[tid] = g;
    if (tid < 2) s_cnt[tid] = 0;
    __syncthreads();
    double el = 0.0;
    const long long t = gp * L + l;
    // Poisson draws grouped by sampler branch: the block's inversion tasks
    // (mu < 10) fill the task list from the front, the others from the back,
    // so that each wave but one runs a single branch
    int cls = -1;
    if (active && set >= 0) {
        double sum = 0.0;
        for (int k = 0; k < L; ++k) sum = sum + g_s[lp * L + k];
        el = (double)pt.e * (g / sum);
        if (el >= P.min_e && el > 0.0) {
            const double mu = el / (double)P.scale;
            s_mu[tid] = mu;
            s_pin[tid] = pin;
            s_evg[tid] = evg;
            cls = mu < 10.0 ? 0 : 1;
            if (cls == 0) s_list[atomicAdd(&s_cnt[0], 1)] = (uint16_t)tid;
            else s_list[kBlock - 1 - atomicAdd(&s_cnt[1], 1)] = (uint16_t)tid;
        }
    }
    __syncthreads();
    {
        const int c0 = s_cnt[0], c1 = s_cnt[1];
        if (tid < c0 + c1) {
            const int task = tid < c0 ? s_list[tid] : s_list[kBlock - 1 - (tid - c0)];
            long long k = poisson_draw<0>(s_mu[task], P.key0, P.key1, (uint32_t)(task % L), s_pin[task],
                                       s_evg[task]);
            if (k < 1) k = 1;
            if (k > P.cap) k = P.cap;
            s_n[task] = (int)k;
        }
    }
    __syncthreads();
    int n = 0;
    float ehit = 0.0f;
    if (cls >= 0) n = s_n[tid];
    if (active && set >= 0) {
        double e_used = el;
        if (G(P.elayer_override)) {
            const float ov = G(P.elayer_override)[t];
            const bool ok = ov >= 0.0f && isfinite(ov);
            if (!ok) gor(&G(P.ctr)->error, (int)kErrOverride);
            e_used = ok ? (double)ov : 0.0;
        }
        ehit = n > 0 ? (float)(e_used / (double)n) : 0.0f;
        // an override below FLT_MIN x n would give subnormal hit energies,
        // which the deposits' count of new cells cannot take
        if (ehit > 0.0f && ehit < P.ehit_min) {
            gor(&G(P.ctr)->error, (int)kErrOverride);
            ehit = 0.0f;
        }
    }
    if (active) {
        G(P.task_n)[t] = n;
        G(P.task_ehit)[t] = ehit;
        if (P.win_path) G(P.task_nT)[(long long)l * P.n_particles + gp] = task_pair(n, ehit);
        if (G(P.out_elayer)) G(P.out_elayer)[t] = (float)el;
        if (G(P.out_counts)) G(P.out_counts)[t] = n;
        if (l == 0) {
            G(P.part_ev)[gp] = ev;
            G(P.part_p)[gp] = pin;
            G(P.part_set)[gp] = set;
        }
    }
    // this block's sums of (hits, chunks, small hits, small tasks) for the
    // task scan (one scan block per workgroup)
    int4 tot;
    (void)block_excl_scan4(active ? task_terms(P, n) : make_int4(0, 0, 0, 0), tot);
    if (tid == 0) store_i4(reinterpret_cast<int4*>(P.blk_sums), blockIdx.x, tot);
}

// A setup workgroup takes `setup_sub` scan blocks of kBlock / L particles
// (at most kSetupPartCap particles, kSetupTaskCap tasks).  Each lane works
// through the tasks tid, tid + kBlock, ... one Gamma attempt per step, so a
// wave waits for its slowest lane's total number of attempts rather than for
// the slowest draw of every task in turn.
constexpr int kSetupSubMax = 4;
constexpr int kSetupTaskCap = kSetupSubMax * kBlock;
constexpr int kSetupPartCap = kBlock;

// Six waves per SIMD (at most 80 VGPRs): the FP64 samplers of large batches
// are throughput-bound, and the extra waves outweigh the larger call frames.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_setup(
    const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    __shared__ double s_g[kSetupTaskCap];       // Gamma draws, then layer energies
    __shared__ double s_mu[kSetupTaskCap];      // Poisson means
    uint32_t* s_w = reinterpret_cast<uint32_t*>(s_mu);  // before them: the boost words
    __shared__ int s_n[kSetupTaskCap];          // hit counts
    __shared__ uint16_t s_list[kSetupTaskCap];  // tasks by Poisson branch
    __shared__ uint32_t s_pin[kSetupPartCap], s_evg[kSetupPartCap];
    __shared__ int s_set[kSetupPartCap];
    __shared__ float s_e[kSetupPartCap];
    __shared__ int s_cnt[2];
    __shared__ int s_pool;  // the Gamma loop's next unclaimed task
    const int L = P.n_layers;
    const int ppb = kBlock / L;
    const int sub = P.setup_sub;
    const int tid = threadIdx.x;
    const long long p0 = (long long)blockIdx.x * ppb * sub;
    const int np = (int)min((long long)(ppb * sub), P.n_particles - p0);
    const int nt = np * L;
    if (P.validate) check_offsets(P);
    if (blockIdx.x == 0 && tid == 0) G(P.queue)[kWinTicket * kQueueStride] = 0;  // the window pass's ticket
    for (int lp = tid; lp < np; lp += kBlock) {
        const long long gp = p0 + lp;
        const Particle pt = load_particle(P.particles, gp);
        if (P.validate) {
            const int err = particle_errors(pt);
            if (err) gor(&G(P.ctr)->error, err);
        }
        const int ev = find_event(G(P.ev_off), P.n_events, P.part_base + gp);
        const uint32_t pin = (uint32_t)(P.part_base + gp - G(P.ev_off)[ev]);
        const uint32_t evg = (uint32_t)(P.ev_base + (unsigned long long)ev);
        note_event_size(P, ev, pin);
        const int set = select_set(P, pt.pdg, pt.e, pt.eta);
        s_set[lp] = set;
        s_pin[lp] = pin;
        s_evg[lp] = evg;
        s_e[lp] = pt.e;
        G(P.part_ev)[gp] = ev;
        G(P.part_p)[gp] = pin;
        G(P.part_set)[gp] = set;
    }
    if (tid < 2) s_cnt[tid] = 0;
    if (tid == 0) s_pool = kBlock;
    __syncthreads();
    {
        // Each lane starts on task tid; a lane whose task is done (accepted,
        // or its 64 attempts spent) takes the workgroup's next unclaimed one,
        // so the lanes stay busy until the pool is empty whatever the
        // rejections.  A task's draws depend only on its counters.
        const int lane = lane_id();
        int t = tid;
        double d = 0.0, c = 0.0;
        uint32_t j = 0;
        bool fresh = true;  // t is a new task: its constants are due
        while (__ballot(t < nt) != 0) {
            bool finished = false;
            if (t < nt) {
                const int lp = t / L;
                const int set = s_set[lp];
                if (set < 0) {  // particles without a set: g = 0
                    s_g[t] = 0.0;
                    finished = true;
                } else {
                    if (fresh) {
                        const double alpha = (double)G(P.alpha)[(set / (P.n_ebins * P.n_etabins)) * L + t % L];
                        const double a = alpha < 1.0 ? alpha + 1.0 : alpha;
                        d = a - 1.0 / 3.0;
                        c = 1.0 / sqrt(9.0 * d);
                        j = 0;
                        fresh = false;
                    }
                    double g = 0.0;
                    uint32_t w = 0;
                    const bool done = gamma_try<1>(d, c, j, P.key0, P.key1, (uint32_t)(t % L), s_pin[lp],
                                                   s_evg[lp], &g, &w);
                    const bool fallback = !done && ++j == 64;
                    if (done || fallback) {
                        // the boost of alpha < 1 waits for the pass below, so
                        // that a wave runs it once for all its lanes
                        s_g[t] = fallback ? d : g;
                        s_w[t] = w;
                        s_n[t] = fallback ? 1 : 0;
                        finished = true;
                    }
                }
            }
            // the finished lanes claim the next tasks, one LDS atomic per wave
            const unsigned long long fm = __ballot(finished);
            if (fm) {
                const int leader = __ffsll((long long)fm) - 1;
                int base = 0;
                if (lane == leader) base = atomicAdd(&s_pool, __popcll(fm));
                base = __shfl(base, leader, kWave);
                if (finished) {
                    t = base + __popcll(fm & ((1ull << lane) - 1ull));
                    fresh = true;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSetupSubMax; ++k) {
        const int t = tid + k * kBlock;
        if (t < nt && s_set[t / L] >= 0 && s_n[t] == 0) {
            const double alpha = (double)G(P.alpha)[(s_set[t / L] / (P.n_ebins * P.n_etabins)) * L + t % L];
            s_g[t] = gamma_boost<1>(s_g[t], alpha, s_w[t]);
        }
    }
    __syncthreads();
    // layer energies (each task sums its particle's draws in layer order);
    // Poisson draws grouped by sampler branch: inversion tasks (mu < 10)
    // fill the list from the front, the others from the back
    double el_t[kSetupSubMax];
#pragma unroll
    for (int k = 0; k < kSetupSubMax; ++k) {
        const int t = tid + k * kBlock;
        el_t[k] = 0.0;
        if (t >= nt) continue;
        const int lp = t / L;
        if (s_set[lp] >= 0) {
            double sum = 0.0;
            for (int q = 0; q < L; ++q) sum = sum + s_g[lp * L + q];
            const double el = (double)s_e[lp] * (s_g[t] / sum);
            el_t[k] = el;
            if (el >= P.min_e && el > 0.0) {
                const double mu = el / (double)P.scale;
                s_mu[t] = mu;
                if (mu < 10.0) s_list[atomicAdd(&s_cnt[0], 1)] = (uint16_t)t;
                else s_list[kSetupTaskCap - 1 - atomicAdd(&s_cnt[1], 1)] = (uint16_t)t;
            }
        }
        s_n[t] = 0;
    }
    if (tid == 0) s_pool = 0;  // the Gamma loop is over: the pool now hands out rejection draws
    __syncthreads();  // every sum has read the draws: they make way for the layer energies
#pragma unroll
    for (int k = 0; k < kSetupSubMax; ++k)
        if (tid + k * kBlock < nt) s_g[tid + k * kBlock] = el_t[k];
    {
        const int c0 = s_cnt[0], c1 = s_cnt[1];
        // inversion draws (mu < 10), one per lane at a time
        for (int i = tid; i < c0; i += kBlock) {
            const int t = s_list[i];
            const int lp = t / L;
            long long k = poisson_draw<1>(s_mu[t], P.key0, P.key1, (uint32_t)(t % L), s_pin[lp], s_evg[lp]);
            if (k < 1) k = 1;
            if (k > P.cap) k = P.cap;
            s_n[t] = (int)k;
        }
        // transformed-rejection draws (mu >= 10): the same attempts in the
        // same order as poisson_draw, taken one step at a time per lane so
        // that the costly parts run with many lanes at once: idle lanes
        // claim new draws (and compute their constants) together once half
        // the wave is idle; an attempt that passes neither quick test waits
        // for the full test until a quarter of the wave waits too, or no
        // lane has a quick step left
        const int lane = lane_id();
        int t = -1;  // the lane's task, -1 when idle
        double mu = 0.0, b = 0.0, a = 0.0, vr = 0.0, log_ia = 0.0, loglam = 0.0;
        double kd = 0.0, us = 0.0, V = 0.0;
        uint32_t att = 0;  // attempt 2j + h: words (x, y) or (z, w) of counter j
        bool full = false; // attempt att awaits the full test
        bool drained = false;
        const auto finish = [&](long long k) {
            if (k < 1) k = 1;
            if (k > P.cap) k = P.cap;
            s_n[t] = (int)k;
            t = -1;
        };
        for (;;) {
            const unsigned long long idle = __ballot(t < 0);
            if (!drained && __popcll(idle) >= kWave / 2) {
                const int leader = __ffsll((long long)idle) - 1;
                int base = 0;
                if (lane == leader) base = atomicAdd(&s_pool, __popcll(idle));
                base = __shfl(base, leader, kWave);
                drained = base + __popcll(idle) >= c1;
                const int k = base + __popcll(idle & ((1ull << lane) - 1ull));
                if (t < 0 && k < c1) {
                    t = s_list[kSetupTaskCap - 1 - k];
                    mu = s_mu[t];
                    const double slam = sqrt(mu);
                    loglam = dlog<1>(mu);
                    b = 0.931 + 2.53 * slam;
                    a = -0.059 + 0.02483 * b;
                    const double invalpha = 1.1239 + 1.1328 / (b - 3.4);
                    vr = 0.9277 - 3.6224 / (b - 2.0);
                    log_ia = dlog<1>(invalpha);
                    att = 0;
                    full = false;
                }
            }
            const unsigned long long quick = __ballot(t >= 0 && !full);
            if (quick == 0 && __ballot(t >= 0) == 0) {
                if (drained) break;
                continue;  // fewer than half the lanes were idle: claim now
            }
            if (t >= 0 && !full) {
                const int lp = t / L;
                const U4 x = philox4x32_10(att >> 1, (uint32_t)(t % L) | (kTagPoisson << 8), s_pin[lp], s_evg[lp],
                                           P.key0, P.key1);
                const uint32_t wu = (att & 1) ? x.z : x.x;
                const uint32_t wv = (att & 1) ? x.w : x.y;
                const double U = unit_open(wu) - 0.5;
                V = unit_open(wv);
                us = 0.5 - fabs(U);
                kd = floor((((2.0 * a) / us + b) * U + mu) + 0.43);
                if (us >= 0.07 && V <= vr) finish((long long)kd);
                else if (kd < 0.0 || (us < 0.013 && V > us)) {
                    if (++att == 64) finish((long long)floor(mu));
                } else {
                    full = true;
                }
            }
            const unsigned long long fm = __ballot(t >= 0 && full);
            if (fm != 0 && (__popcll(fm) >= kWave / 4 || __ballot(t >= 0 && !full) == 0)) {
                if (t >= 0 && full) {
                    const double lhs = (dlog<1>(V) + log_ia) - dlog<1>(a / (us * us) + b);
                    const double rhs = (-mu + kd * loglam) - dlnfact<1>((long long)kd);
                    full = false;
                    if (lhs <= rhs) finish((long long)kd);
                    else if (++att == 64) finish((long long)floor(mu));
                }
            }
        }
    }
    __syncthreads();
    for (int t = tid; t < nt; t += kBlock) {
        const int lp = t / L, l = t - lp * L;
        const long long gt = (p0 + lp) * L + l;
        const int n = s_n[t];
        const double el = s_g[t];
        const int set = s_set[lp];
        float ehit = 0.0f;
        if (set >= 0) {
            double e_used = el;
            if (G(P.elayer_override)) {
                const float ov = G(P.elayer_override)[gt];
                const bool ok = ov >= 0.0f && isfinite(ov);
                if (!ok) gor(&G(P.ctr)->error, (int)kErrOverride);
                e_used = ok ? (double)ov : 0.0;
            }
            ehit = n > 0 ? (float)(e_used / (double)n) : 0.0f;
            if (ehit > 0.0f && ehit < P.ehit_min) {
                gor(&G(P.ctr)->error, (int)kErrOverride);
                ehit = 0.0f;
            }
        }
        G(P.task_n)[gt] = n;
        G(P.task_ehit)[gt] = ehit;
        if (G(P.out_elayer)) G(P.out_elayer)[gt] = (float)el;
        if (G(P.out_counts)) G(P.out_counts)[gt] = n;
        if (P.win_path) s_w[t] = __float_as_uint(ehit);
    }
    // the window pass reads (hits, Ehit) layer-major: consecutive lanes
    // write consecutive particles of one layer
    if (P.win_path) {
        __syncthreads();
        for (int k = tid; k < nt; k += kBlock) {
            const int l = k / np, lp = k - l * np;
            const int t = lp * L + l;
            G(P.task_nT)[(long long)l * P.n_particles + p0 + lp] = task_pair(s_n[t], __uint_as_float(s_w[t]));
        }
    }
    // the task scan's sums of (hits, chunks, small hits, small tasks), one
    // wave per scan block of this workgroup
    const int lane = lane_id();
    for (int sb = tid / kWave; sb < sub; sb += kBlock / kWave) {
        int4 acc = make_int4(0, 0, 0, 0);
        for (int q = lane; q < ppb * L; q += kWave) {
            const int t = sb * ppb * L + q;
            if (t < nt) acc = add4(acc, task_terms(P, s_n[t]));
        }
#pragma unroll
        for (int dd = kWave / 2; dd > 0; dd >>= 1) {
            acc.x += __shfl_xor(acc.x, dd, kWave);
            acc.y += __shfl_xor(acc.y, dd, kWave);
            acc.z += __shfl_xor(acc.z, dd, kWave);
            acc.w += __shfl_xor(acc.w, dd, kWave);
        }
        const long long b = (long long)blockIdx.x * sub + sb;
        if (lane == 0 && b < P.n_scan_blocks) store_i4(reinterpret_cast<int4*>(P.blk_sums), b, acc);
    }
}

// ----------------------------------------- task scans -> work queue (a11) ---
// per task: x = hits, y = chunks of a large task, z = hits of a small task,
// w = 1 for a small task with hits

// The task scan runs over the setup blocks' sums in two levels.  Groups of
// kGroupItems block sums are scanned by one 1024-thread block each (loads and
// stores coalesced, staged through LDS); one block then scans the group
// totals.  Hits are summed in 64 bits (more than 2^31 - 1 hits in a batch is
// an error, found in the top pass); the other components are bounded by the
// task count.
constexpr int kScanThreads = 1024;
constexpr int kGroupPer = 2;                              // block sums per thread
constexpr int kGroupItems = kScanThreads * kGroupPer;     // block sums per group

// exclusive scan over a 1024-thread block of (hits, rest): returns the
// thread's exclusive prefix and the block totals
__device__ __forceinline__ void scan1024(long long h, int4 r, long long& ho, int4& ro, long long& htot,
                                         int4& rtot)
{
    constexpr int kW = kScanThreads / kWave;
    __shared__ long long w_hits[kW];
    __shared__ int4 w_rest[kW];
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const long long hi = wave_incl_scan<long long>(h);
    const int4 ri = wave_incl_scan4(r);
    if (lane == kWave - 1) {
        w_hits[wave] = hi;
        w_rest[wave] = ri;
    }
    __syncthreads();
    ho = hi - h;
    ro = sub4(ri, r);
    htot = 0;
    rtot = make_int4(0, 0, 0, 0);
    for (int w = 0; w < kW; ++w) {
        const long long wh = w_hits[w];
        const int4 wr = w_rest[w];
        if (w < wave) {
            ho += wh;
            ro = add4(ro, wr);
        }
        htot += wh;
        rtot = add4(rtot, wr);
    }
    __syncthreads();
}

// batch totals of the task scan into the counters (errors for too many hits
// or too many chunks) and the work-queue tickets reset; called by every
// thread of the block that finishes the scan
__device__ __forceinline__ void scan_totals(const Params& P, long long htot, int4 rtot)
{
    const int tid = threadIdx.x;
    // the hit kernel's tickets and drained flags (the window pass's ticket is
    // reset by the setup pass: the window pass may already be running)
    if (tid < kWinTicket) G(P.queue)[tid * kQueueStride] = 0;
    if (tid == 0) {
        auto cc = G(P.ctr);
        cc->hits_total = htot;
        int err = 0;
        if (htot > 2147483647LL) err |= kErrTooManyHits;
        if (rtot.y > P.chunk_cap) {
            err |= kErrChunkCap;
            cc->need_chunks = rtot.y;
        }
        cc->n_chunks = err ? 0 : rtot.y;
        cc->n_small_hits = err ? 0 : rtot.z;
        cc->n_small_tasks = err ? 0 : rtot.w;
        cc->n_tiles = err ? 0 : (int)(((long long)rtot.z + P.tile_hits - 1) / P.tile_hits);
        if (err) gor(&cc->error, err);
        if (G(P.out_task_hoff) && !err) G(P.out_task_hoff)[P.n_tasks] = P.hit_base + htot;
    }
}

// one block per group: exclusive prefixes of the group's block sums (hits
// in 32 bits, valid whenever the batch total is) and the group's totals;
// with a single group it also finishes the scan
__global__ __launch_bounds__(kScanThreads) void k_scan_group(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    __shared__ int4 s_v[kGroupItems];
    const int tid = threadIdx.x;
    const long long base = (long long)blockIdx.x * kGroupItems;
    const long long nb = P.n_scan_blocks;
    const int4* in = reinterpret_cast<const int4*>(P.blk_sums);
    int4* out = reinterpret_cast<int4*>(P.blk_offs);
#pragma unroll
    for (int k = 0; k < kGroupPer; ++k) {
        const long long b = base + k * kScanThreads + tid;
        s_v[k * kScanThreads + tid] = b < nb ? load_i4(in, b) : make_int4(0, 0, 0, 0);
    }
    __syncthreads();
    int4 v[kGroupPer];
    long long h = 0;
    int4 r = make_int4(0, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < kGroupPer; ++k) {
        v[k] = s_v[tid * kGroupPer + k];
        h += v[k].x;
        r = add4(r, make_int4(0, v[k].y, v[k].z, v[k].w));
    }
    long long ho, htot;
    int4 ro, rtot;
    scan1024(h, r, ho, ro, htot, rtot);
#pragma unroll
    for (int k = 0; k < kGroupPer; ++k) {
        s_v[tid * kGroupPer + k] = make_int4((int)ho, ro.y, ro.z, ro.w);
        ho += v[k].x;
        ro = add4(ro, make_int4(0, v[k].y, v[k].z, v[k].w));
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kGroupPer; ++k) {
        const long long b = base + k * kScanThreads + tid;
        if (b < nb) store_i4(out, b, s_v[k * kScanThreads + tid]);
    }
    if (tid == 0) {
        G(P.grp_hits)[blockIdx.x] = htot;
        store_i4(reinterpret_cast<int4*>(P.grp_rest), blockIdx.x, rtot);
    }
    // a batch of one group needs no top pass
    if (P.n_scan_groups == 1) {
        if (tid == 0) store_i4(reinterpret_cast<int4*>(P.grp_offs), 0, make_int4(0, 0, 0, 0));
        scan_totals(P, htot, rtot);
    }
}

// one block: exclusive scan of the group totals into the group offsets;
// batch totals into the counters, work-queue tickets reset
__global__ __launch_bounds__(kScanThreads) void k_scan_top(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const int tid = threadIdx.x;
    const int ng = P.n_scan_groups;
    const int per = (ng + kScanThreads - 1) / kScanThreads;
    const int g0 = tid * per;
    const int4* rest = reinterpret_cast<const int4*>(P.grp_rest);
    int4* out = reinterpret_cast<int4*>(P.grp_offs);
    long long h = 0;
    int4 r = make_int4(0, 0, 0, 0);
    for (int k = 0; k < per; ++k) {
        const int g = g0 + k;
        if (g < ng) {
            h += G(P.grp_hits)[g];
            const int4 q = load_i4(rest, g);
            r = add4(r, make_int4(0, q.y, q.z, q.w));
        }
    }
    long long ho, htot;
    int4 ro, rtot;
    scan1024(h, r, ho, ro, htot, rtot);
    for (int k = 0; k < per; ++k) {
        const int g = g0 + k;
        if (g < ng) {
            store_i4(out, g, make_int4((int)ho, ro.y, ro.z, ro.w));
            ho += G(P.grp_hits)[g];
            const int4 q = load_i4(rest, g);
            ro = add4(ro, make_int4(0, q.y, q.z, q.w));
        }
    }
    scan_totals(P, htot, rtot);
}

// one thread per task, over the setup blocks (particles kBlock / L at a
// time): the task's place in the hit list, its chunks, its small-task
// records and the first task of every tile it opens
__global__ __launch_bounds__(kBlock) void k_scan_write(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    if (G(P.ctr)->error & (kErrTooManyHits | kErrChunkCap)) return;
    const int L = P.n_layers;
    const int ppb = kBlock / L;
    const int tid = threadIdx.x;
    const long long t = (long long)blockIdx.x * ppb * L + tid;
    const bool active = tid < ppb * L && t < P.n_tasks;
    const int n = active ? G(P.task_n)[t] : 0;
    const int4 d = task_terms(P, n);
    int4 tot;
    const int4 run = add4(add4(block_excl_scan4(d, tot),
                               load_i4(reinterpret_cast<const int4*>(P.blk_offs), blockIdx.x)),
                          load_i4(reinterpret_cast<const int4*>(P.grp_offs), blockIdx.x / kGroupItems));
    if (!active) return;
    if (P.want_hits) G(P.task_hoff)[t] = run.x;
    if (G(P.out_task_hoff)) G(P.out_task_hoff)[t] = P.hit_base + run.x;
    const long long gp = t / L;
    const int key = (int)(gp * 64 + (t - gp * L));
    for (int c = 0; c < d.y; ++c) {
        const int first = c * P.chunk_hits;
        const int cnt = min(P.chunk_hits, n - first);
        store_i4(P.chunks, run.y + c, make_int4(key, first, cnt, 0));
    }
    if (d.w && !P.win_path) {
        // two 16-byte records per small task: (first small hit, task key,
        // Ehit bits, histogram) and (eta_p, phi_p, global event, particle
        // in event)
        const Particle pt = load_particle(P.particles, gp);
        const int H = G(P.part_set)[gp] * L + (key & 63);
        store_i4(P.small_rec, 2LL * run.w,
                 make_int4(run.z, key, __float_as_int(G(P.task_ehit)[t]), H));
        const uint32_t evg = (uint32_t)(P.ev_base + (unsigned long long)G(P.part_ev)[gp]);
        store_i4(P.small_rec, 2LL * run.w + 1,
                 make_int4(__float_as_int(pt.eta), __float_as_int(pt.phi), (int)evg,
                           (int)G(P.part_p)[gp]));
        const int T = P.tile_hits;
        const int q = (run.z + T - 1) / T;
        if ((long long)q * T < (long long)run.z + n) G(P.tile_first)[q] = run.w;
    }
}

// ------------------------------------------------------ the hit (a4 - a7) ---
// Geometry tables, built at load time and staged in LDS by every workgroup
// of the hit kernels (as int vectors; float fields travel as their bits):
//   layer l,  3 records: (acc_lo, acc_hi, inv_r, -), eta_lo of regions 0..3,
//                        eta_lo of regions 4..7 (+inf past the last region)
//   region r, 2 records: (eta_lo, inv_deta, phi_lo, inv_dphi),
//                        (neta, nphi, first cell, -)
struct GeoLds {
    const v4i* layers;
    const v4i* regions;
    int n_regions;
};

__device__ __forceinline__ float f_of(int v) { return __int_as_float(v); }

// The three records of a layer (acceptance and 1/R; region lower edges).
struct LayerRec {
    v4i a, b0, b1;
};

__device__ __forceinline__ LayerRec layer_rec(const GeoLds& g, int l)
{
    return LayerRec{g.layers[3 * l], g.layers[3 * l + 1], g.layers[3 * l + 2]};
}

// region-grid lookup (Listing 2's getDDE): -1 outside the acceptance
// [eta_lo(first region), eta_hi(last region)); the region is the number of
// interior region edges <= eta (only the layer's n_regions - 1 real edges are
// compared); cell indices are clamped into the grid
__device__ __forceinline__ int lookup_cell(const GeoLds& g, const LayerRec& lr, int l, float eta,
                                           float phi)
{
    if (!(eta >= f_of(lr.a.x)) || !(eta < f_of(lr.a.y))) return -1;
    // edges past the last region are +inf and never counted; layers of at
    // most four regions (a uniform branch) compare only the first three
    int k = (int)(eta >= f_of(lr.b0.y)) + (int)(eta >= f_of(lr.b0.z)) + (int)(eta >= f_of(lr.b0.w));
    if (g.n_regions > 4)
        k += (int)(eta >= f_of(lr.b1.x)) + (int)(eta >= f_of(lr.b1.y)) + (int)(eta >= f_of(lr.b1.z)) +
             (int)(eta >= f_of(lr.b1.w));
    const int r = l * g.n_regions + k;
    const v4i f = g.regions[2 * r];
    const v4i iv = g.regions[2 * r + 1];
    int ie = (int)floorf((eta - f_of(f.x)) * f_of(f.y));
    int ip = (int)floorf((phi - f_of(f.z)) * f_of(f.w));
    ie = min(max(ie, 0), iv.x - 1);
    ip = min(max(ip, 0), iv.y - 1);
    // 0 <= ie * nphi < n_cells <= 2^28: a full-rate 24-bit multiply
    return iv.z + (int)__umul24((unsigned)ie, (unsigned)iv.y) + ip;
}

// The same lookup in FP64 (FP64 placement variant): the position compared
// and scaled in FP64 against the FP32 geometry values.
__device__ __forceinline__ int lookup_cell_f64(const GeoLds& g, const LayerRec& lr, int l,
                                               double eta, double phi)
{
    if (!(eta >= (double)f_of(lr.a.x)) || !(eta < (double)f_of(lr.a.y))) return -1;
    int k = (int)(eta >= (double)f_of(lr.b0.y)) + (int)(eta >= (double)f_of(lr.b0.z)) +
            (int)(eta >= (double)f_of(lr.b0.w));
    if (g.n_regions > 4)
        k += (int)(eta >= (double)f_of(lr.b1.x)) + (int)(eta >= (double)f_of(lr.b1.y)) +
             (int)(eta >= (double)f_of(lr.b1.z)) + (int)(eta >= (double)f_of(lr.b1.w));
    const int r = l * g.n_regions + k;
    const v4i f = g.regions[2 * r];
    const v4i iv = g.regions[2 * r + 1];
    int ie = (int)floor((eta - (double)f_of(f.x)) * (double)f_of(f.y));
    int ip = (int)floor((phi - (double)f_of(f.z)) * (double)f_of(f.w));
    ie = min(max(ie, 0), iv.x - 1);
    ip = min(max(ip, 0), iv.y - 1);
    return iv.z + ie * iv.y + ip;
}

// stage the geometry tables into LDS (call with every thread, then sync)
__device__ __forceinline__ GeoLds stage_geometry(const Params& P, v4i* s_geo)
{
    const int nl = 3 * P.n_layers;
    const int nr = 2 * P.n_layers * P.n_regions;
    const FCS_AS_GLOBAL v4i* gl = (const FCS_AS_GLOBAL v4i*)P.geo_layers;
    const FCS_AS_GLOBAL v4i* gr = (const FCS_AS_GLOBAL v4i*)P.geo_regions;
    for (int i = threadIdx.x; i < nl; i += blockDim.x) s_geo[i] = gl[i];
    for (int i = threadIdx.x; i < nr; i += blockDim.x) s_geo[nl + i] = gr[i];
    return GeoLds{s_geo, s_geo + nl, P.n_regions};
}

// first bin with cum > u; the guide narrows the search to [g[j], g[j+1]]
// (g[kGuide] = kBins - 1).  kPadded: the guide holds that last entry, as
// the per-wave LDS copies do; else both reads stay inside the histogram's
// kGuide entries and the last one is selected.
template <bool kPadded, typename CumT, typename GuideT>
__device__ __forceinline__ int find_bin(CumT cum, GuideT guide, uint32_t x0, float u)
{
    const int j = (int)(x0 >> 22);  // u0 = (x0 >> 8) 2^-24 lies in [j, j+1) / kGuide
    int lo = guide[j];
    int hi;
    if constexpr (kPadded) {
        hi = guide[j + 1];
    } else {
        const int g1 = guide[j < kGuide - 1 ? j + 1 : j];
        hi = j < kGuide - 1 ? g1 : kBins - 1;
    }
    // cum is nondecreasing, so the bin is lo plus the number of entries of
    // [lo, hi) at or below u.  From global memory (the window pass and the
    // tiles) the usual short ranges read their (at most three) entries at
    // once instead of one dependent read per halving; from LDS the halving
    // loop issues fewer instructions
    if (!kPadded && hi - lo <= 3) {
        const float c0 = cum[lo];
        const float c1 = cum[min(lo + 1, kBins - 1)];
        const float c2 = cum[min(lo + 2, kBins - 1)];
        return lo + (int)(lo < hi && c0 <= u) + (int)(lo + 1 < hi && c1 <= u) + (int)(lo + 2 < hi && c2 <= u);
    }
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cum[mid] > u) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

struct HitOut {
    float eta, phi;
    int cell, bin;
    uint32_t w4;  // the counter's fourth word (the energy fluctuation's uniform)
};

// one hit: counter (i, layer | 3 << 8, particle in event, global event)
// -> three 24-bit uniforms -> (r, alpha) bin -> position in the bin ->
// (eta, phi) -> cell.  kTask: the wave's hits belong to one task (layer,
// particle and event uniform; padded guide in LDS).  kF64: the placement
// and the cell lookup in FP64 (a chain variant; same uniforms and bin).
template <bool kTask, bool kF64 = false, typename CumT, typename GuideT>
__device__ __forceinline__ HitOut simulate_hit(const GeoLds& g, const LayerRec& lr, CumT cum,
                                               GuideT guide, float dr, uint32_t k0, uint32_t k1,
                                               uint32_t i, uint32_t l, uint32_t pin, uint32_t evg,
                                               float eta_p, float phi_p)
{
    const float inv_r = f_of(lr.a.z);
    const U4 x = kTask ? philox4x32_10_uniform_ctr(i, l | (kTagHit << 8), pin, evg, k0, k1)
                       : philox4x32_10(i, l | (kTagHit << 8), pin, evg, k0, k1);
    const float u0 = unit24(x.x), u1 = unit24(x.y), u2 = unit24(x.z);
    HitOut h;
    h.w4 = x.w;
    h.bin = find_bin<kTask>(cum, guide, x.x, u0);
    const int ir = h.bin >> 3, ia = h.bin & 7;
    if constexpr (kF64) {
        // r = (ir + u1) dr and alpha = 2 pi (ia + u2) / 8, both in FP64;
        // cos and sin from the FP64 series in turns (sin at t - 1/4)
        const double rr = ((double)ir + (double)u1) * (double)dr;
        const double t = ((double)ia + (double)u2) * 0.125;
        const double cd = dcos_turns<2>(t);
        const double sd = dcos_turns<2>(t - 0.25);
        const double inv_r64 = (double)inv_r;
        const double eta64 = (double)eta_p + (rr * cd) * inv_r64;
        double phi64 = (double)phi_p + (rr * sd) * inv_r64;
        const double pi64 = 3.14159265358979323846, two_pi64 = 6.28318530717958647692;
        if (phi64 >= pi64) phi64 = phi64 - two_pi64;
        else if (phi64 < -pi64) phi64 = phi64 + two_pi64;
        h.eta = (float)eta64;
        h.phi = (float)phi64;
        h.cell = lookup_cell_f64(g, lr, (int)l, eta64, phi64);
        return h;
    }
    const float r = __builtin_fmaf(u1, dr, (float)ir * dr);  // lower edge + u1 * dr, one rounding
    float c, s;
    sincos_bin(ia, u2, c, s);
    const float deta = (r * c) * inv_r;
    const float dphi = (r * s) * inv_r;
    const float eta = eta_p + deta;
    float phi = phi_p + dphi;
    const float pi_f = 3.14159265358979323846f;
    const float two_pi_f = 6.28318530717958647692f;
    // one wrap into [-pi_f, pi_f), both candidates computed, no branch
    const float lo = phi - two_pi_f, hi = phi + two_pi_f;
    phi = phi >= pi_f ? lo : (phi < -pi_f ? hi : phi);
    h.eta = eta;
    h.phi = phi;
    h.cell = lookup_cell(g, lr, (int)l, eta, phi);
    return h;
}

__device__ __forceinline__ void write_hit(const Params& P, long long pos, const HitOut& h, float e)
{
    pos += P.hit_base;
    if (pos < P.hit_cap) {
        G(P.hit_eta)[pos] = h.eta;
        G(P.hit_phi)[pos] = h.phi;
        G(P.hit_e)[pos] = e;
        G(P.hit_cell)[pos] = h.cell;
    }
}

// Uniform description of one chunk of a large (particle, layer) task.
struct ChunkInfo {
    int t, l, first, count, ev, H;
    uint32_t pin, evg;
    float ehit, eta_p, phi_p;
};

__device__ __forceinline__ ChunkInfo load_chunk(const Params& P, int item)
{
    const int4 ck = load_i4(P.chunks, item);
    ChunkInfo c;
    const int key = __builtin_amdgcn_readfirstlane(ck.x);
    c.first = __builtin_amdgcn_readfirstlane(ck.y);
    c.count = __builtin_amdgcn_readfirstlane(ck.z);
    const int gp = key >> 6;
    c.l = key & 63;
    c.t = gp * P.n_layers + c.l;
    c.ehit = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(G(P.task_ehit)[c.t])));
    c.ev = __builtin_amdgcn_readfirstlane(G(P.part_ev)[gp]);
    c.pin = (uint32_t)__builtin_amdgcn_readfirstlane((int)G(P.part_p)[gp]);
    c.evg = (uint32_t)(P.ev_base + (unsigned long long)c.ev);
    c.H = __builtin_amdgcn_readfirstlane(G(P.part_set)[gp]) * P.n_layers + c.l;
    const Particle pt = load_particle(P.particles, gp);
    c.eta_p = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(pt.eta)));
    c.phi_p = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(pt.phi)));
    return c;
}

// ------------------------------------------------------ wave-level items ---
// Every wave of the hit kernels runs its own work items (no workgroup
// barriers inside the item loop); the LDS below is partitioned per wave.
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kWaveSlots = 512;  // LDS hash slots of one wave's chunk accumulator
constexpr int kListCap = 512;    // per-wave u16 tile-owner list (in the hash key array)
static_assert(kTileMax <= kListCap, "a tile's owners must fit the owner list");
static_assert(kListCap * 2 <= kWaveSlots * 4 && kListCap * 2 <= kBins * 8,
              "the owner list borrows a wave's hash keys or bin sums");
static_assert(kGuide / 16 == kWave && kBins / 4 == kWave, "one 16-byte record per lane");
static_assert(kChunkMax < 65536, "per-cell chunk counts are 16-bit");
static_assert(kWaveSlots == 512, "hash_bits caps the table at 2^9 slots");
// per-step (event, cell) table of the tile path: 64-bit keys in the wave's
// guide area, FP32 sums in its histogram area (both reloaded per chunk)
constexpr int kTileBits = 7;
constexpr int kTileSlots = 1 << kTileBits;
static_assert(kTileSlots * 8 <= kGuide && kTileSlots * 4 <= kBins * 4 && kTileSlots >= 2 * kWave,
              "the tile table borrows a wave's guide and histogram");
constexpr unsigned long long kEmpty64 = ~0ull;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}


// Owners of the hits of a tile of small tasks, for one wave: every task that
// starts inside the tile marks its first hit with its index relative to the
// tile's first task; an inclusive max-scan fills the gaps.  T <= kListCap.
__device__ __forceinline__ void wave_tile_owners(const Params& P, const FCS_AS_GLOBAL Counters* ctr,
                                                 int q, uint16_t* owner, int& s0, int& h0,
                                                 int& hcount)
{
    const int lane = lane_id();
    const int T = P.tile_hits;
    h0 = q * T;
    hcount = min(T, ctr->n_small_hits - h0);
    s0 = G(P.tile_first)[q];
    const int s1 = (q + 1 < ctr->n_tiles) ? G(P.tile_first)[q + 1] : ctr->n_small_tasks - 1;
    for (int k = lane; k < T; k += kWave) owner[k] = 0;
    wave_sync();
    for (int j = s0 + lane; j <= s1; j += kWave) {
        int st = load_i4(P.small_rec, 2LL * j).x - h0;
        st = st < 0 ? 0 : st;
        if (st < T) owner[st] = (uint16_t)(j - s0);
    }
    wave_sync();
    const int per = T / kWave;  // consecutive entries per lane
    int m = 0;
    for (int k = 0; k < per; ++k) {
        const int v = owner[lane * per + k];
        m = v > m ? v : m;
    }
    int inc = m;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int o = __shfl_up(inc, d, kWave);
        if (lane >= d) inc = o > inc ? o : inc;
    }
    int run = __shfl_up(inc, 1, kWave);
    if (lane == 0) run = 0;
    for (int k = 0; k < per; ++k) {
        const int v = owner[lane * per + k];
        run = v > run ? v : run;
        owner[lane * per + k] = (uint16_t)run;
    }
    wave_sync();
}

// Per-hit description of a hit of a small task (from its two records).
struct SmallHit {
    int t, l, i, ev, H;
    uint32_t pin, evg;
    float ehit, eta_p, phi_p;
};

__device__ __forceinline__ SmallHit small_hit(const Params& P, int j, int hit)
{
    const int4 r0 = load_i4(P.small_rec, 2LL * j);
    const int4 r1 = load_i4(P.small_rec, 2LL * j + 1);
    SmallHit s;
    s.i = hit - r0.x;
    const int gp = r0.y >> 6;
    s.l = r0.y & 63;
    s.t = gp * P.n_layers + s.l;
    s.ehit = __int_as_float(r0.z);
    s.H = r0.w;
    s.eta_p = __int_as_float(r1.x);
    s.phi_p = __int_as_float(r1.y);
    s.evg = (uint32_t)r1.z;
    s.pin = (uint32_t)r1.w;
    s.ev = (int)(s.evg - (uint32_t)P.ev_base);
    return s;
}

// Deposit into an event's cell and keep the per-64-cell-block count of
// nonzero cells (one byte per block, packed four to a word): the adder that
// finds the cell at zero counts it.  Energies are positive, so exactly one
// adder sees zero.
__device__ __forceinline__ float deposit_add(const Params& P, long long ev, int cell, float v)
{
    const auto cp = G(P.cells) + ev * P.n_cells + cell;
    float old;
    [[clang::atomic(ignore_denormal_mode)]] {
        old = __hip_atomic_fetch_add(cp, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return old;
}

// the count word of (event, cell) and the increment of the cell's block in it
__device__ __forceinline__ FCS_AS_GLOBAL uint32_t* count_word(const Params& P, long long ev, int cell)
{
    const long long b = ev * P.n_blk + (cell >> 6);
    return (FCS_AS_GLOBAL uint32_t*)(G(P.flags) + (b & ~3LL));
}
__device__ __forceinline__ uint32_t count_inc(int cell) { return 1u << (8 * ((cell >> 6) & 3)); }

__device__ __forceinline__ void deposit(const Params& P, long long ev, int cell, float v)
{
    if (!(v > 0.0f)) return;  // zero-energy hits leave the cell untouched
    if (deposit_add(P, ev, cell, v) == 0.0f) (void)gfetch_add(count_word(P, ev, cell), count_inc(cell));
}

// Claim or find the slot of `key` in a wave's tile table (linear probing);
// true for the lane that claimed it.  A step inserts at most kWave keys into
// kTileSlots >= 2 kWave slots, so a free or matching slot is always found.
__device__ __forceinline__ bool tile_slot(unsigned long long* tkey, unsigned long long key, uint32_t h,
                                          int& slot)
{
    slot = (int)(h >> (32 - kTileBits));
    for (int pr = 0; pr < kTileSlots; ++pr) {
        const unsigned long long o = atomicCAS(&tkey[slot], kEmpty64, key);
        if (o == kEmpty64) return true;
        if (o == key) return false;
        slot = (slot + 1) & (kTileSlots - 1);
    }
    return false;
}

__device__ __forceinline__ uint32_t tile_hash(uint32_t a, uint32_t b)
{
    return (a * 0x9E3779B1u) ^ (b * 0x85EBCA77u);
}

// add `cnt` hits of `key` to a wave's LDS hash table (linear probing over
// the first 2^bits slots; two 16-bit counts per word, a chunk has at most
// kChunkMax hits); when no slot is found the energy goes to the cell directly
__device__ __forceinline__ void wave_hash_add(const Params& P, uint32_t* hkey, uint32_t* hcnt2,
                                              int bits, uint32_t key, uint32_t cnt, long long ev,
                                              float ehit)
{
    const uint32_t mask = (1u << bits) - 1u;
    // multiplicative hash on the key's low 24 bits with the full-rate 24-bit
    // multiplier (v_mul_u32_u24; a 32-bit v_mul_lo_u32 is quarter rate).
    // __umul24 returns a signed int: the product is taken as unsigned before
    // the shift, so the slot stays in [0, 2^bits).
    uint32_t slot = (uint32_t)__umul24(key, 0x9E3779u) >> (32 - bits);
    for (int pr = 0; pr < kHashProbes; ++pr) {
        const uint32_t old = atomicCAS(&hkey[slot], kEmpty, key);
        if (old == kEmpty || old == key) {
            atomicAdd(&hcnt2[slot >> 1], cnt << (16 * (slot & 1)));
            return;
        }
        slot = (slot + 1) & mask;
    }
    deposit(P, ev, (int)key, (float)cnt * ehit);
}

// hash slots used for a chunk of n hits: about 2n (at most half full), 64 to
// kWaveSlots, so that a small chunk's flush reads few words
__device__ __forceinline__ int hash_bits(int n)
{
    const int b = 32 - __clz(2 * n - 1);  // ceil(log2(2n))
    return b < 6 ? 6 : (b > 9 ? 9 : b);
}

// deposit every claimed slot among the first 2^bits of a wave's table as
// count * Ehit and clear it (call with the whole wave after a wave_sync)
__device__ __forceinline__ void wave_hash_flush(const Params& P, uint32_t* hkey, uint32_t* hcnt2,
                                                int bits, long long ev, float ehit)
{
    for (int w = lane_id(); w < (1 << (bits - 1)); w += kWave) {
        const uint32_t c2 = hcnt2[w];
        if (c2 == 0) continue;
        const uint32_t lo = c2 & 0xffffu, hi = c2 >> 16;
        if (lo) {
            deposit(P, ev, (int)hkey[2 * w], (float)lo * ehit);
            hkey[2 * w] = kEmpty;
        }
        if (hi) {
            deposit(P, ev, (int)hkey[2 * w + 1], (float)hi * ehit);
            hkey[2 * w + 1] = kEmpty;
        }
        hcnt2[w] = 0;
    }
}

// ------------------------------------------- per-hit energy fluctuation ---
// A chain variant: the hit's energy is Ehit x with x = -ln u exponential
// (mean 1), u = ((w4 >> 8) + 1/2) 2^-24 from the counter's fourth word, x in
// FP64 with the setup's log series, one rounding to FP32.
__device__ __forceinline__ double fluct_factor(uint32_t w4)
{
    const double u = ((double)(w4 >> 8) + 0.5) * 0x1p-24;
    return -dlog<2>(u);
}

__device__ __forceinline__ float fluct_energy(float ehit, uint32_t w4)
{
    return (float)((double)ehit * fluct_factor(w4));
}

// the chunk path's hash with FP64 energy sums per slot (the variant's
// energies differ per hit, so counts x Ehit do not apply)
__device__ __forceinline__ void wave_hash_add_e(const Params& P, uint32_t* hkey, double* hsum,
                                                int bits, uint32_t key, float e, long long ev)
{
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t slot = (uint32_t)__umul24(key, 0x9E3779u) >> (32 - bits);
    for (int pr = 0; pr < kHashProbes; ++pr) {
        const uint32_t old = atomicCAS(&hkey[slot], kEmpty, key);
        if (old == kEmpty || old == key) {
            atomicAdd(&hsum[slot], (double)e);
            return;
        }
        slot = (slot + 1) & mask;
    }
    deposit(P, ev, (int)key, e);
}

__device__ __forceinline__ void wave_hash_flush_e(const Params& P, uint32_t* hkey, double* hsum,
                                                  int bits, long long ev)
{
    for (int k = lane_id(); k < (1 << bits); k += kWave) {
        const uint32_t key = hkey[k];
        if (key == kEmpty) continue;
        deposit(P, ev, (int)key, (float)hsum[k]);
        hkey[k] = kEmpty;
        hsum[k] = 0.0;
    }
}

// ----------------------------------------------------------- work queue ---
// The items are split into kQueues contiguous ranges with one ticket counter
// each.  A wave starts on the range of its workgroup's slot (workgroups are
// dispatched round-robin over the chip's 8 XCDs, so neighbouring items, which
// share events and cells, tend to stay in one XCD's L2) and takes per_grab
// items per ticket; when its range is drained it moves on to the next.  One
// counter handing out single items would serialize every wave on one atomic.
struct WaveQueue {
    int n_items, per_grab, home, probe, cur, end;
};

// workgroups of a persistent grid that the items can keep busy (at least one
// item per wave); the others leave before staging anything
__device__ __forceinline__ int active_workgroups(int n_items)
{
    const int need = (n_items + kWavesPerBlock - 1) / kWavesPerBlock;
    return need < (int)gridDim.x ? need : (int)gridDim.x;
}

__device__ __forceinline__ WaveQueue make_queue(int n_items, int active_wg)
{
    WaveQueue q;
    q.n_items = n_items;
    const long long waves = (long long)active_wg * (blockDim.x / kWave);
    const long long k = n_items / (waves * 16);
    q.per_grab = (int)(k < 1 ? 1 : (k > 32 ? 32 : k));
    q.home = (int)(blockIdx.x & (kQueues - 1));
    q.probe = 0;
    q.cur = q.end = 0;
    return q;
}

// next item for the calling wave (uniform), false once every range is drained
__device__ __forceinline__ bool next_item(const Params& P, WaveQueue& q, int& item)
{
    if (q.cur < q.end) {
        item = q.cur++;
        return true;
    }
    const auto tickets = G(P.queue);
    const auto drained = G(P.queue) + kQueues * kQueueStride;
    while (q.probe < kQueues) {
        const int r = (q.home + q.probe) & (kQueues - 1);
        ++q.probe;
        // a plain load of the range's drained flag spares most late atomics
        if (__builtin_amdgcn_readfirstlane(drained[r * kQueueStride])) continue;
        const int lo = (int)((long long)r * q.n_items / kQueues);
        const int hi = (int)((long long)(r + 1) * q.n_items / kQueues);
        int g = 0;
        if (lane_id() == 0) g = gfetch_add(tickets + r * kQueueStride, q.per_grab);
        g = __builtin_amdgcn_readfirstlane(g);
        if (lo + g < hi) {
            item = lo + g;
            q.cur = item + 1;
            q.end = min(item + q.per_grab, hi);
            q.probe = 0;  // come back to the home range first next time
            return true;
        }
        if (lane_id() == 0) drained[r * kQueueStride] = 1;
    }
    return false;
}

// ------------------------------------------------- persistent hit kernel ---
// Work items, pulled by each wave from a ticket counter: [0, n_chunks)
// chunks of large (particle, layer) tasks, then tiles of packed small tasks.
// A chunk's histogram and guide are staged in the wave's LDS; its hits are
// counted per cell in the wave's LDS hash table (the lanes that share the cell
// of a leading lane are counted together first, once per step) and flushed
// once as count * Ehit, one rounding per cell and chunk.  Tile hits that share an
// (event, cell) with a leading lane are summed across the wave first; each
// remaining sum goes to the event's cell with one device atomic.
// kTiles: the instantiation that also deposits the packed tiles of small
// tasks (the window pass takes them otherwise; without that path the chunk
// loop has the registers to itself)
template <bool kF64, bool kFluct, bool kTiles = true>
__global__ __launch_bounds__(kBlock) void k_hits(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    extern __shared__ v4i s_geo[];
    __shared__ uint32_t w_key[kWavesPerBlock][kWaveSlots];
    __shared__ uint32_t w_cnt2[kWavesPerBlock][kWaveSlots / 2];
    // energy fluctuation variant: FP64 energy sums per hash slot
    __shared__ double w_esum[kFluct ? kWavesPerBlock : 1][kFluct ? kWaveSlots : 1];
    __shared__ float w_cum[kWavesPerBlock][kBins];
    __shared__ v4i w_guide16[kWavesPerBlock][kGuide / 16 + 1];  // + the pad entry

    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    uint32_t* hkey = w_key[wv];
    uint32_t* hcnt2 = w_cnt2[wv];
    double* hsum = w_esum[kFluct ? wv : 0];
    uint16_t* owners = reinterpret_cast<uint16_t*>(hkey);  // tiles only
    float* cum = w_cum[wv];
    const uint8_t* guide = reinterpret_cast<const uint8_t*>(w_guide16[wv]);
    unsigned long long* tkey = reinterpret_cast<unsigned long long*>(w_guide16[wv]);  // tiles only
    float* tval = w_cum[wv];                                                           // tiles only
    uint32_t* tinc = reinterpret_cast<uint32_t*>(w_cum[wv]);                           // tiles only

    const auto ctr = G(P.ctr);
    if (ctr->error & (kErrTooManyHits | kErrChunkCap)) return;
    const int n_chunks = ctr->n_chunks;
    // with the window pass the small tasks are deposited by k_windows
    const int n_items = n_chunks + (P.win_path ? 0 : ctr->n_tiles);
    const int active_wg = active_workgroups(n_items);
    if ((int)blockIdx.x >= active_wg) return;
    const float dr = P.r_max / 32.0f;
    const uint32_t k0 = P.key0, k1 = P.key1;
    long long n_out = 0;

    const GeoLds geo = stage_geometry(P, s_geo);
    for (int s = lane; s < kWaveSlots; s += kWave) hkey[s] = kEmpty;
    for (int s = lane; s < kWaveSlots / 2; s += kWave) hcnt2[s] = 0;
    if constexpr (kFluct)
        for (int s = lane; s < kWaveSlots; s += kWave) hsum[s] = 0.0;
    if (lane == 0) reinterpret_cast<uint8_t*>(w_guide16[wv])[kGuide] = kBins - 1;  // the pad entry
    __syncthreads();

    WaveQueue queue = make_queue(n_items, active_wg);
    int item;
    while (next_item(P, queue, item)) {

        if (item < n_chunks) {
            // ------------------------------------------- chunk of a large task
            const ChunkInfo ck = load_chunk(P, item);
            const long long hb = (long long)ck.H * kBins;
            reinterpret_cast<v4i*>(cum)[lane] = ((const FCS_AS_GLOBAL v4i*)(G(P.cum) + hb))[lane];
            w_guide16[wv][lane] = ((const FCS_AS_GLOBAL v4i*)(G(P.guide) + (long long)ck.H * kGuide))[lane];
            wave_sync();
            const LayerRec lrec = layer_rec(geo, ck.l);
            const int hbits = hash_bits(ck.count);
            const long long hbase = P.want_hits ? (long long)G(P.task_hoff)[ck.t] : 0;
            for (int i = ck.first + lane; i < ck.first + ck.count; i += kWave) {
                const HitOut h = simulate_hit<true, kF64>(geo, lrec, cum, guide, dr, k0, k1, (uint32_t)i,
                                              (uint32_t)ck.l, ck.pin, ck.evg, ck.eta_p, ck.phi_p);
                n_out += h.cell < 0 ? 1 : 0;
                if constexpr (kFluct) {
                    const float e = fluct_energy(ck.ehit, h.w4);
                    if (P.want_hits) write_hit(P, hbase + i, h, e);
                    if (h.cell >= 0) wave_hash_add_e(P, hkey, hsum, hbits, (uint32_t)h.cell, e, ck.ev);
                    continue;
                }
                if (P.want_hits) write_hit(P, hbase + i, h, ck.ehit);
                // the lanes in the first valid lane's cell (often the shower
                // core) are counted by that lane's insert, which runs beside
                // the other lanes' inserts of one hit each
                const bool valid = h.cell >= 0;
                const unsigned long long act = __ballot(valid);
                if (act) {
                    const int leader = __ffsll((long long)act) - 1;
                    const int lk = __builtin_amdgcn_readlane(h.cell, leader);
                    const bool same = valid && h.cell == lk;
                    const unsigned long long sm = __ballot(same);
                    if (lane == leader || (valid && !same))
                        wave_hash_add(P, hkey, hcnt2, hbits, (uint32_t)h.cell,
                                      lane == leader ? (uint32_t)__popcll(sm) : 1u, ck.ev, ck.ehit);
                }
            }
            wave_sync();
            if constexpr (kFluct) wave_hash_flush_e(P, hkey, hsum, hbits, ck.ev);
            else wave_hash_flush(P, hkey, hcnt2, hbits, ck.ev, ck.ehit);
            wave_sync();
        } else if constexpr (kTiles) {
            // ------------------------------------------ tile of small tasks
            int s0, h0, hcount;
            wave_tile_owners(P, ctr, item - n_chunks, owners, s0, h0, hcount);
            // uniform trip count: every lane takes part in the wave sums below
            for (int kb = 0; kb < hcount; kb += kWave) {
                const int k = kb + lane;
                const bool valid = k < hcount;
                const int kk = valid ? k : hcount - 1;
                const SmallHit sh = small_hit(P, s0 + owners[kk], h0 + kk);
                const HitOut h = simulate_hit<false, kF64>(geo, layer_rec(geo, sh.l),
                                              G(P.cum) + (long long)sh.H * kBins,
                                              G(P.guide) + (long long)sh.H * kGuide, dr, k0, k1,
                                              (uint32_t)sh.i, (uint32_t)sh.l, sh.pin, sh.evg,
                                              sh.eta_p, sh.phi_p);
                const float e_hit = kFluct ? fluct_energy(sh.ehit, h.w4) : sh.ehit;
                if (valid && P.want_hits)
                    write_hit(P, (long long)G(P.task_hoff)[sh.t] + sh.i, h, e_hit);
                n_out += (valid && h.cell < 0) ? 1 : 0;
                // The step's hits are summed per (event, cell) in the wave's
                // LDS table; the lane that claims a slot deposits its sum, so
                // each (event, cell) of the step costs one device atomic.
                tkey[lane] = kEmpty64;
                tkey[lane + kWave] = kEmpty64;
                tval[lane] = 0.0f;
                tval[lane + kWave] = 0.0f;
                wave_sync();
                bool owner = false;
                int slot = 0;
                if (valid && h.cell >= 0) {
                    owner = tile_slot(tkey, ((unsigned long long)(uint32_t)sh.ev << 32) | (uint32_t)h.cell,
                                      tile_hash((uint32_t)h.cell, (uint32_t)sh.ev), slot);
                    atomicAdd(&tval[slot], e_hit);
                }
                wave_sync();
                const float v = owner ? tval[slot] : 0.0f;
                const bool fresh = v > 0.0f && deposit_add(P, sh.ev, h.cell, v) == 0.0f;
                // the step's new cells are counted per count word (four
                // blocks) in the same table: one device atomic per word
                wave_sync();
                tkey[lane] = kEmpty64;
                tkey[lane + kWave] = kEmpty64;
                tinc[lane] = 0u;
                tinc[lane + kWave] = 0u;
                wave_sync();
                bool wowner = false;
                if (fresh) {
                    wowner = tile_slot(tkey, ((unsigned long long)(uint32_t)sh.ev << 32) | ((uint32_t)h.cell >> 8),
                                       tile_hash((uint32_t)h.cell >> 8, (uint32_t)sh.ev), slot);
                    atomicAdd(&tinc[slot], count_inc(h.cell));
                }
                wave_sync();
                if (wowner) (void)gfetch_add(count_word(P, sh.ev, h.cell), tinc[slot]);
                wave_sync();
            }
            wave_sync();
            // the owner list borrowed the hash keys: empty them again
            for (int k = lane; k < kWaveSlots; k += kWave) hkey[k] = kEmpty;
            wave_sync();
        }
    }
    const long long tot = block_sum_ll(n_out);
    if (threadIdx.x == 0 && tot) (void)gfetch_add(&G(P.ctr)->hits_out, tot);
}

// --------------------------------- small tasks by cell window (a8, a11) ---
// Events of many particles (hard scatter, pile-up) put most of their hits in
// (particle, layer) tasks of a few hits each, scattered over the event's
// cells; depositing them with one device atomic per distinct cell of a tile
// step is bound by the memory-side atomic unit, which handles one cache line
// per operation.  This pass instead takes, per work item, one event, one
// window of at most kWinCells consecutive cells of one layer and a range of
// win_parts particles: the small tasks of those particles in that layer are
// simulated (particles whose hits cannot reach the window are skipped), the
// hits landing in the window are summed in a dense LDS copy of it, and the
// touched rows are added to the event's cells with coalesced atomics (64
// consecutive cells per wave instruction, 16 per cache line).  Hits are
// counted out of acceptance, and written to the hit list, by the particle's
// home window (the one whose eta band holds it) only.
constexpr int kWinThreads = 512;
constexpr int kWinWaves = kWinThreads / kWave;
constexpr int kWinCells = 8192;   // 32 KB of LDS: three workgroups per CU
constexpr int kWinPerCu = 3;      // resident workgroups of the window pass per CU
constexpr int kFlushWords = 4;    // count words (1,024 cells) per wave and flush round
static_assert(kWinCells % 64 == 0, "windows are whole 64-cell rows of LDS");

// window record, two int4 per window: (layer, first cell, end cell, index of
// the layer's first window), (eta band low, eta band high (float bits),
// windows of the layer, -)
struct WinRec {
    int layer, c_lo, c_hi, first;
    float b_lo, b_hi;
    int n_layer;
};

// from the copy staged in LDS after the geometry records
__device__ __forceinline__ WinRec load_window(const v4i* s_win, int w)
{
    const v4i a = s_win[2 * w];
    const v4i b = s_win[2 * w + 1];
    return WinRec{a.x, a.y, a.z, a.w, __int_as_float(b.x), __int_as_float(b.y), b.z};
}

__global__ __launch_bounds__(kWinThreads) void k_windows(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    extern __shared__ v4i s_geo[];
    __shared__ float s_acc[kWinCells];
    __shared__ int s_st[kWinThreads];     // per wave: first position of each staged task's hits
    // per wave and round: owner marks, slot numbers below 64 (zero between
    // rounds); bytes, so that three workgroups still fit a CU's LDS
    __shared__ uint8_t s_mark[kWinThreads];
    __shared__ v4i s_pa[kWinThreads];     // (histogram | home << 31, Ehit, eta, phi)
    __shared__ int2 s_pb[kWinThreads];    // (particle in event, task)
    __shared__ int s_item;
    __shared__ int s_next;                // next group of 64 particles of the item's range

    const auto ctr = G(P.ctr);
    if (!P.win_path || (ctr->error & (kErrTooManyHits | kErrChunkCap))) return;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const int L = P.n_layers;
    const long long E = P.n_events;
    const long long n_cells = P.n_cells;
    const int max_np = ctr->max_event_particles;
    const int n_pr = (max_np + P.win_parts - 1) / P.win_parts;  // particle ranges per event
    const long long n_items = (long long)P.n_windows * E * n_pr;
    if (n_items == 0) return;
    const float dr = P.r_max / 32.0f;
    const uint32_t k0 = P.key0, k1 = P.key1;
    long long n_out = 0;

    const GeoLds geo = stage_geometry(P, s_geo);
    // the window records follow the geometry records in the dynamic LDS
    v4i* s_win = s_geo + 3 * P.n_layers + 2 * P.n_layers * P.n_regions;
    for (int i = tid; i < 2 * P.n_windows; i += kWinThreads) s_win[i] = ((const FCS_AS_GLOBAL v4i*)P.geo_windows)[i];
    for (int c = tid; c < kWinCells; c += kWinThreads) s_acc[c] = 0.0f;
    s_mark[tid] = 0;
    const auto ticket = G(P.queue) + kWinTicket * kQueueStride;
    if (tid == 0) s_item = gfetch_add(ticket, 1);
    for (;;) {
        if (tid == 0) s_next = 0;  // every wave has left the previous item's groups
        __syncthreads();  // the previous item's flush is complete; s_item is set
        const long long item = s_item;
        __syncthreads();  // every thread has read it
        if (item >= n_items) break;
        // the next item's ticket is taken now, its latency hidden behind this one
        if (tid == 0) s_item = gfetch_add(ticket, 1);
        // window-major order: the windows of the first layers (the most hits)
        // are handed out first
        const int r = (int)(item % n_pr);
        const long long e = (item / n_pr) % E;
        const int w = (int)(item / ((long long)n_pr * E));
        const WinRec win = load_window(s_win, w);
        const int l = win.layer;
        const LayerRec lrec = layer_rec(geo, l);
        // particles of this launch in event e, this item's range of them
        const long long ev0 = G(P.ev_off)[e] - P.part_base, ev1 = G(P.ev_off)[e + 1] - P.part_base;
        const long long a = ev0 + (long long)r * P.win_parts;
        const long long b = min(ev1, a + (long long)P.win_parts);
        if (a >= b) continue;
        const uint32_t evg = (uint32_t)(P.ev_base + (unsigned long long)e);
        // a hit lands at most r_max / R_l away in eta (margins for rounding)
        const float reach = P.r_max * f_of(lrec.a.z) * 1.001f + 1e-3f;
        // each wave claims groups of 64 particles of the range until none is
        // left: it stages their tasks in its 64 slots, scans them within the
        // wave and simulates their hits 64 at a time (a task's hits on
        // consecutive lanes); the waves meet only before the flush
        const int wbase = wave * kWave;
        for (;;) {
            int g = 0;
            if (lane == 0) g = atomicAdd(&s_next, kWave);
            const long long pg = a + __builtin_amdgcn_readfirstlane(g);
            if (pg >= b) break;
            const long long p = pg + lane;
            int n = 0;
            if (p < b) {
                const long long t = p * L + l;
                // the particle's records are loaded beside its task's pair
                // (one memory round trip per group, not two), used or not
                const unsigned long long ne = G(P.task_nT)[(long long)l * P.n_particles + p];
                const Particle pt = load_particle(P.particles, p);
                const int pset = G(P.part_set)[p];
                const int ppin = (int)G(P.part_p)[p];
                const int nt = (int)(uint32_t)ne;
                if (nt > 0 && nt < P.big_thr) {
                    // home window: the one of this layer whose band holds eta
                    int home = win.first;
                    for (int k = win.first; k < win.first + win.n_layer - 1; ++k) {
                        const WinRec wk = load_window(s_win, k);
                        home += pt.eta >= wk.b_hi ? 1 : 0;
                    }
                    const bool is_home = home == w;
                    if (is_home || (pt.eta >= win.b_lo - reach && pt.eta <= win.b_hi + reach)) {
                        n = nt;
                        const int H = pset * L + l;
                        s_pa[tid] = v4i{H | (is_home ? (int)0x80000000u : 0), (int)(uint32_t)(ne >> 32),
                                        __float_as_int(pt.eta), __float_as_int(pt.phi)};
                        s_pb[tid] = make_int2(ppin, (int)t);
                    }
                }
            }
            // the wave's staged hits in slot order: slot j holds [st, inc)
            const int inc = wave_scan_dpp<false>(n);
            const int total = __builtin_amdgcn_readlane(inc, kWave - 1);
            const int st = inc - n;
            s_st[tid] = st;
            for (int q0 = 0; q0 < total; q0 += kWave) {
                // owner of hit q0 + k: every slot with hits in [q0, q0 + 64)
                // marks its first position there (distinct positions, the
                // slot holding q0 at position 0), a max-scan fills the gaps
                if (n > 0 && st < q0 + kWave && inc > q0) s_mark[wbase + (st > q0 ? st - q0 : 0)] = (uint8_t)lane;
                wave_sync();
                const int own = wave_scan_dpp<true>((int)s_mark[tid]);
                s_mark[tid] = 0;
                const int q = q0 + lane;
                if (q < total) {
                    const int j = wbase + own;
                    const int i = q - s_st[j];  // hit index within its task
                    const v4i pa = s_pa[j];
                    const int2 pbk = s_pb[j];
                    const int H = pa.x & 0x7fffffff;
                    const float ehit = __int_as_float(pa.y);
                    const HitOut h = simulate_hit<false>(geo, lrec, G(P.cum) + (long long)H * kBins,
                                                         G(P.guide) + (long long)H * kGuide, dr, k0, k1,
                                                         (uint32_t)i, (uint32_t)l, (uint32_t)pbk.x, evg,
                                                         __int_as_float(pa.z), __int_as_float(pa.w));
                    if (h.cell >= win.c_lo && h.cell < win.c_hi) atomicAdd(&s_acc[h.cell - win.c_lo], ehit);
                    if (pa.x < 0) {  // home window
                        n_out += h.cell < 0 ? 1 : 0;
                        if (P.want_hits) write_hit(P, (long long)G(P.task_hoff)[pbk.y] + i, h, ehit);
                    }
                }
            }
            wave_sync();  // the wave's slots are restaged by its next group
        }
        __syncthreads();  // every wave's hits are in the accumulator
        // flush the window: each wave takes kFlushWords count words (four
        // 64-cell blocks of the event's cells each) per round, issues the
        // coalesced atomic adds of all their nonzero rows, and only then
        // reads the returned values: the adds that find a cell at zero count
        // it, one count-word atomic per word
        {
            constexpr int kFW = kFlushWords, kR = 4 * kFlushWords;
            const long long g0 = win.c_lo, g1 = win.c_hi;  // [g0, g1)
            const auto cells = G(P.cells) + e * n_cells;
            const long long wlast = (g1 - 1) >> 8;
            for (long long wd = (g0 >> 8) + (long long)wave * kFW; wd <= wlast; wd += (long long)kWinWaves * kFW) {
                float v[kR], old[kR];
#pragma unroll
                for (int k = 0; k < kR; ++k) {
                    const long long g = wd * 256 + k * 64 + lane;
                    const bool in = g >= g0 && g < g1;
                    const float a = s_acc[in ? (int)(g - g0) : 0];
                    v[k] = in ? a : 0.0f;
                }
#pragma unroll
                for (int k = 0; k < kR; ++k) {
                    old[k] = 1.0f;
                    if (v[k] != 0.0f) {
                        const long long g = wd * 256 + k * 64 + lane;
                        [[clang::atomic(ignore_denormal_mode)]] {
                            old[k] = __hip_atomic_fetch_add(cells + g, v[k], __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                        }
                        s_acc[g - g0] = 0.0f;
                    }
                }
#pragma unroll
                for (int q = 0; q < kFW; ++q) {
                    uint32_t word = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        word |= (uint32_t)__popcll(__ballot(old[4 * q + k] == 0.0f)) << (8 * k);
                    if (lane == 0 && word)
                        (void)gfetch_add(
                            (FCS_AS_GLOBAL uint32_t*)(G(P.flags) + ((e << P.blk_shift) + (wd + q) * 4)), word);
                }
            }
        }
    }
    const long long tot = block_sum_ll<kWinThreads>(n_out);
    if (threadIdx.x == 0 && tot) (void)gfetch_add(&G(P.ctr)->hits_out, tot);
}

// ------------------------------------- per-(particle, layer) launches ---
// The launch form of the paper's first GPU port, kept as a baseline: one
// launch per (particle, layer) task with one thread per hit.  The hit is the
// same function of its counter as in k_hits; the task's histogram is read
// from global memory.  All hits of a task carry the same energy, so each
// workgroup counts its hits per cell in LDS and adds count x Ehit to the
// cell with one device atomic (one rounding per cell and workgroup, as the
// chunk path flushes; a device atomic per hit would round once per hit),
// keeping the per-block counts of nonzero cells for the compaction.
constexpr int kTaskSlots = 2 * kBlock;  // LDS cell slots of a workgroup
static_assert(kTaskSlots == 512, "the slot hash takes 9 bits");

template <bool kF64, bool kFluct>
__global__ __launch_bounds__(kBlock) void k_task_hits(const Params* __restrict__ Pp, int t)
{
    const Params& P = *Pp;
    extern __shared__ v4i s_geo[];
    __shared__ int s_cell[kTaskSlots];
    __shared__ uint32_t s_cnt[kTaskSlots];
    __shared__ double s_esum[kFluct ? kTaskSlots : 1];  // energy fluctuation variant
    if (G(P.ctr)->error & (kErrTooManyHits | kErrChunkCap)) return;
    const GeoLds geo = stage_geometry(P, s_geo);
    for (int k = threadIdx.x; k < kTaskSlots; k += kBlock) {
        s_cell[k] = -1;
        s_cnt[k] = 0u;
        if constexpr (kFluct) s_esum[k] = 0.0;
    }
    __syncthreads();
    const int L = P.n_layers;
    const int gp = t / L, l = t - gp * L;
    const int n = G(P.task_n)[t];
    const int i = (int)blockIdx.x * kBlock + (int)threadIdx.x;
    const int ev = G(P.part_ev)[gp];
    const float ehit = G(P.task_ehit)[t];
    long long n_out = 0;
    if (i < n) {
        const int H = G(P.part_set)[gp] * L + l;
        const uint32_t pin = (uint32_t)G(P.part_p)[gp];
        const uint32_t evg = (uint32_t)(P.ev_base + (unsigned long long)ev);
        const Particle pt = load_particle(P.particles, gp);
        const HitOut h = simulate_hit<false, kF64>(geo, layer_rec(geo, l), G(P.cum) + (long long)H * kBins,
                                             G(P.guide) + (long long)H * kGuide, P.r_max / 32.0f,
                                             P.key0, P.key1, (uint32_t)i, (uint32_t)l, pin, evg,
                                             pt.eta, pt.phi);
        const float e_hit = kFluct ? fluct_energy(ehit, h.w4) : ehit;
        if (P.want_hits) write_hit(P, (long long)G(P.task_hoff)[t] + i, h, e_hit);
        if (h.cell < 0) {
            n_out = 1;
        } else {
            // linear probing; at most kBlock distinct cells in kTaskSlots slots
            uint32_t k = ((uint32_t)h.cell * 2654435761u) >> (32 - 9);
            for (;;) {
                const int prev = atomicCAS(&s_cell[k], -1, h.cell);
                if (prev == -1 || prev == h.cell) break;
                k = (k + 1) & (kTaskSlots - 1);
            }
            atomicAdd(&s_cnt[k], 1u);
            if constexpr (kFluct) atomicAdd(&s_esum[k], (double)e_hit);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kTaskSlots; k += kBlock)
        if (s_cnt[k]) deposit(P, ev, s_cell[k], kFluct ? (float)s_esum[k] : (float)s_cnt[k] * ehit);
    const long long tot = block_sum_ll(n_out);
    if (threadIdx.x == 0 && tot) (void)gfetch_add(&G(P.ctr)->hits_out, tot);
}

// ---------------------------------------------------- asynchronous calls ---
// one thread: fold the call's counters and capacity checks into the
// context's running totals (stream order serializes the calls)
__device__ __forceinline__ void fold_async(const Params& P, AsyncAcc* acc, bool count_call, long long nnz)
{
    const auto c = G(P.ctr);
    int err = c->error;
    if (G(P.out_ids) && nnz > P.out_cap) err |= kErrCellCap;
    if (P.want_hits && c->hits_total > P.hit_cap) err |= kErrHitCap;
    const auto a = G(acc);
    if (count_call) {  // simulation calls; adjoint calls fold their errors only
        a->n_calls += 1;
        a->hits += c->hits_total;
        a->hits_out += c->hits_out;
        a->nnz += nnz;
    }
    a->error |= err;
}

// ---------------------------------------------- range-checked loads ---
// Raw buffer loads: a load at a byte offset at or beyond the resource's size
// returns 0 and reads no memory, so a batch of loads needs no branch (and no
// wait between its loads) to skip unused slots.  Word 3 selects the 32-bit
// data format of the gfx9 family.
constexpr int kBufWord3 = 0x00020000;
constexpr uint32_t kBufNone = 0xFFFFFFF0u;  // an offset beyond every resource here

__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kBufWord3);
}

__device__ inline float buf_load_f32(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

__device__ inline long long buf_load_i64(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(long long, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// ------------------------------------------ ordered compaction (a10) ---
// The hit kernels keep, per event and 64-cell block, the number of nonzero
// cells (one byte per block).  A wave per segment of 1024 blocks (16 per
// lane) counts its nonzero cells and nonzero blocks; a scan over segments
// gives every nonzero block its place in a block list and the output
// position of its first nonzero cell, in ascending (event, cell) order.  The
// list pass writes the list and resets the counts; the emit pass takes 16
// listed blocks per wave whatever the events' density, writes the nonzero
// cells as (cell_id, E) and resets them.
constexpr int kSegBlocks = 1024;
constexpr int kEmitBatch = 16;
static_assert(kSegBlocks == 16 * kWave, "a lane holds 16 block counts");

__device__ __forceinline__ int byte_sum(uint32_t w)
{
    return (int)(w & 0xff) + (int)((w >> 8) & 0xff) + (int)((w >> 16) & 0xff) + (int)(w >> 24);
}

__device__ __forceinline__ int byte_nonzero(uint32_t w)
{
    return (int)((w & 0xff) != 0) + (int)((w & 0xff00) != 0) + (int)((w & 0xff0000) != 0) +
           (int)((w & 0xff000000u) != 0);
}

__device__ __forceinline__ const FCS_AS_GLOBAL v4i* seg_counts(const Params& P, long long e, int seg)
{
    return (const FCS_AS_GLOBAL v4i*)(G(P.flags) + (e << P.blk_shift) + (long long)seg * kSegBlocks);
}

// Count pass: a workgroup per group of kSegGroup segments, kSegPerWave per
// wave (their loads in flight together).  Per segment the nonzero cells (low
// 32 bits) and nonzero blocks (high 32 bits); the segments' exclusive
// prefixes within the group go to seg_off and the group's total to seg_blk.
constexpr int kSegGroup = kSegPerWave * kWavesPerBlock;
__global__ __launch_bounds__(kBlock) void k_seg_count(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    __shared__ long long s_c[kSegGroup];
    const long long n = P.n_events * P.n_seg;
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const long long g0 = (long long)blockIdx.x * kSegGroup;
    const long long w0 = g0 + wave * kSegPerWave;
    v4i w[kSegPerWave];
#pragma unroll
    for (int k = 0; k < kSegPerWave; ++k) {
        const long long gw = w0 + k;
        w[k] = v4i{0, 0, 0, 0};
        if (gw < n) {
            const long long e = gw / P.n_seg;
            w[k] = seg_counts(P, e, (int)(gw - e * P.n_seg))[lane];
        }
    }
#pragma unroll
    for (int k = 0; k < kSegPerWave; ++k) {
        const uint32_t x = (uint32_t)w[k].x, y = (uint32_t)w[k].y, z = (uint32_t)w[k].z,
                       q = (uint32_t)w[k].w;
        // at most 65,536 cells and 1,024 blocks per segment: both fit one word
        uint32_t c = (uint32_t)(byte_sum(x) + byte_sum(y) + byte_sum(z) + byte_sum(q)) +
                     ((uint32_t)(byte_nonzero(x) + byte_nonzero(y) + byte_nonzero(z) + byte_nonzero(q))
                      << 17);
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) c += __shfl_xor(c, d, kWave);
        if (lane == 0) s_c[wave * kSegPerWave + k] = (long long)(c & 0x1ffffu) + ((long long)(c >> 17) << 32);
    }
    __syncthreads();
    if (wave == 0) {
        const long long v = lane < kSegGroup ? s_c[lane] : 0;
        const long long inc = wave_incl_scan<long long>(v);
        if (lane < kSegGroup && g0 + lane < n) G(P.seg_off)[g0 + lane] = inc - v;
        if (lane == kSegGroup - 1) G(P.seg_blk)[blockIdx.x] = inc;
    }
}

// one block: exclusive scan of the group totals; batch totals (nonzero cells,
// listed blocks) into the counters
__global__ __launch_bounds__(1024) void k_seg_top(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    __shared__ long long carry;
    __shared__ long long part[1024 / kWave];
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    const int nb = P.n_seg_groups;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int b = b0 + tid;
        const long long v = b < nb ? G(P.seg_blk)[b] : 0;
        const long long inc = wave_incl_scan<long long>(v);
        if (lane_id() == kWave - 1) part[tid / kWave] = inc;
        __syncthreads();
        long long off = 0, tot = 0;
        for (int w = 0; w < 1024 / kWave; ++w) {
            if (w < tid / kWave) off += part[w];
            tot += part[w];
        }
        if (b < nb) G(P.seg_blk)[b] = carry + off + inc - v;
        __syncthreads();
        if (tid == 0) carry += tot;
        __syncthreads();
    }
    if (tid == 0) {
        const long long nnz = carry & 0xffffffffLL;
        G(P.ctr)->nnz_total = nnz;
        G(P.ctr)->n_blk_list = carry >> 32;
        if (G(P.out_ev_off)) G(P.out_ev_off)[P.n_events] = P.out_base + nnz;
        // every counter and error bit of the call is final here (the passes
        // after this one set none)
        if (P.fold_acc) fold_async(P, P.fold_acc, true, nnz);
    }
}

// list pass: a wave per segment writes an entry per nonzero block (global
// block id, output position of its first nonzero cell) and resets the counts
__global__ __launch_bounds__(kBlock) void k_seg_list(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const long long gw = (long long)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (gw >= P.n_events * P.n_seg) return;
    const long long e = gw / P.n_seg;
    const int seg = (int)(gw - e * P.n_seg);
    const int lane = lane_id();
    const auto w4p = const_cast<FCS_AS_GLOBAL v4i*>(seg_counts(P, e, seg));
    const v4i w = w4p[lane];
    const uint32_t words[4] = {(uint32_t)w.x, (uint32_t)w.y, (uint32_t)w.z, (uint32_t)w.w};
    const int cells = byte_sum(words[0]) + byte_sum(words[1]) + byte_sum(words[2]) + byte_sum(words[3]);
    const int blocks = byte_nonzero(words[0]) + byte_nonzero(words[1]) + byte_nonzero(words[2]) +
                       byte_nonzero(words[3]);
    const long long so = G(P.seg_off)[gw] + G(P.seg_blk)[gw / kSegGroup];
    int pos = (int)(so & 0xffffffffLL) + wave_incl_scan(cells) - cells;
    long long at = (so >> 32) + wave_incl_scan(blocks) - blocks;
    if (seg == 0 && lane == 0 && G(P.out_ev_off)) G(P.out_ev_off)[e] = P.out_base + (so & 0xffffffffLL);
    const uint32_t gb0 = ((uint32_t)e << P.blk_shift) + (uint32_t)(seg * kSegBlocks + lane * 16);
    const auto list = G(P.blk_list);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int cnt = (int)((words[j >> 2] >> (8 * (j & 3))) & 0xffu);
        if (cnt) {
            list[at] = ((unsigned long long)(uint32_t)pos << 32) | (gb0 + (uint32_t)j);
            ++at;
            pos += cnt;
        }
    }
    if (cells) w4p[lane] = v4i{0, 0, 0, 0};
}

// Calls whose only cell output is the caller's dense buffer skip the
// compaction: this pass counts the nonzero cells from the per-block counts
// (the nnz statistic) and clears those counts for the next call.
__global__ __launch_bounds__(kBlock) void k_flags_reset(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const long long n = P.n_events << (P.blk_shift - 4);  // 16-byte words
    auto f = (FCS_AS_GLOBAL v4i*)G(P.flags);
    long long s = 0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        const v4i w = f[i];
        if (w.x | w.y | w.z | w.w) {
            s += byte_sum((uint32_t)w.x) + byte_sum((uint32_t)w.y) + byte_sum((uint32_t)w.z) +
                 byte_sum((uint32_t)w.w);
            f[i] = v4i{0, 0, 0, 0};
        }
    }
    const long long tot = block_sum_ll(s);
    if (threadIdx.x != 0) return;
    if (tot) (void)gfetch_add(&G(P.ctr)->nnz_total, tot);
    if (!P.fold_acc) return;
    // asynchronous calls: the last workgroup to finish folds the call's
    // totals (its ticket is taken after its own count is added)
    __threadfence();
    if (gfetch_add(&G(P.ctr)->done, 1u) == gridDim.x - 1) {
        __threadfence();
        const long long nnz =
            __hip_atomic_load(&G(P.ctr)->nnz_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        fold_async(P, P.fold_acc, true, nnz);
    }
}

// emit pass: persistent waves take kEmitBatch listed blocks at a time; all
// loads of a batch are range-checked buffer loads issued before their use
__global__ __launch_bounds__(kBlock) void k_seg_emit(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    // Parameters used after the first store are kept in registers: the
    // compiler cannot tell the output stores from the parameter block.
    const long long n = G(P.ctr)->n_blk_list;
    const int shift = P.blk_shift;
    const uint32_t bmask = (1u << shift) - 1u;
    const long long n_cells = P.n_cells, out_cap = P.out_cap, out_base = P.out_base;
    const bool clean = P.clean_cells != 0;
    const auto out_ids = G(P.out_ids);
    const auto out_e = G(P.out_e);
    const auto cells0 = G(P.cells);
    const auto list = G(P.blk_list);
    // n_cells <= 2^28, so every byte offset below fits 32 bits
    const auto ids_r = buf_rsrc((const long long*)G(P.cell_id), (uint32_t)(n_cells * 8));
    const int lane = lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    const long long step = (long long)gridDim.x * kWavesPerBlock * kEmitBatch;
    long long b0 = ((long long)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave) * kEmitBatch;
    // the list entries of a wave's next batch are loaded while it works on
    // the current one
    unsigned long long e_next = 0;
    if (lane < kEmitBatch && b0 + lane < n) e_next = list[b0 + lane];
    for (; b0 < n; b0 += step) {
        const unsigned long long e64 = e_next;
        const int2 ent = make_int2((int)(uint32_t)e64, (int)(uint32_t)(e64 >> 32));
        const int nb = (int)(n - b0 < kEmitBatch ? n - b0 : kEmitBatch);
        float v[kEmitBatch];
#pragma unroll
        for (int b = 0; b < kEmitBatch; ++b) {
            const uint32_t gb = (uint32_t)__builtin_amdgcn_readlane(ent.x, b);
            const auto rs = buf_rsrc((const float*)(cells0 + (long long)(gb >> shift) * n_cells),
                                     (uint32_t)(n_cells * 4));
            v[b] = buf_load_f32(rs, b < nb ? ((gb & bmask) * 64u + (uint32_t)lane) * 4u : kBufNone);
        }
        long long id[kEmitBatch];
#pragma unroll
        for (int b = 0; b < kEmitBatch; ++b) {
            const uint32_t gb = (uint32_t)__builtin_amdgcn_readlane(ent.x, b);
            id[b] = buf_load_i64(ids_r, v[b] != 0.0f ? ((gb & bmask) * 64u + (uint32_t)lane) * 8u : kBufNone);
        }
        e_next = 0;
        if (lane < kEmitBatch && b0 + step + lane < n) e_next = list[b0 + step + lane];
#pragma unroll
        for (int b = 0; b < kEmitBatch; ++b) {
            const uint32_t gb = (uint32_t)__builtin_amdgcn_readlane(ent.x, b);
            const int pos = __builtin_amdgcn_readlane(ent.y, b);
            const unsigned long long nz = __ballot(v[b] != 0.0f);
            if (b < nb && v[b] != 0.0f) {
                const long long o = out_base + pos + __popcll(nz & below);
                if (o < out_cap) {
                    out_ids[o] = id[b];
                    out_e[o] = v[b];
                }
                if (clean)
                    cells0[(long long)(gb >> shift) * n_cells + (gb & bmask) * 64u + (uint32_t)lane] = 0.0f;
            }
        }
    }
}

// ------------------------------------------------------ adjoint (a12) ---
// Same work items and wave organization as k_hits.  Each hit's bin and cell
// are recomputed from its Philox counter; g = dL/dE_cell is gathered at the
// cell and accumulated in FP64 per task (sum of g) and per histogram bin (sum
// of g * Ehit); a chunk keeps its 256 bin sums in the wave's LDS and flushes
// them once.
// kFluct: the per-hit energy fluctuation variant; a hit carries E_l x / n, so
// it adds g x to its task's sum and g E_hit to its bin's.
template <bool kFluct>
__global__ __launch_bounds__(kBlock) void k_adjoint(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    extern __shared__ v4i s_geo[];
    __shared__ double w_bin[kWavesPerBlock][kBins];
    __shared__ float w_cum[kWavesPerBlock][kBins];
    __shared__ v4i w_guide16[kWavesPerBlock][kGuide / 16 + 1];  // + the pad entry

    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    double* bins = w_bin[wv];
    uint16_t* owners = reinterpret_cast<uint16_t*>(bins);  // tiles only
    float* cum = w_cum[wv];
    const uint8_t* guide = reinterpret_cast<const uint8_t*>(w_guide16[wv]);
    const auto ctr = G(P.ctr);
    if (ctr->error & (kErrTooManyHits | kErrChunkCap)) return;
    const int n_chunks = ctr->n_chunks;
    const int n_items = n_chunks + ctr->n_tiles;
    const int active_wg = active_workgroups(n_items);
    if ((int)blockIdx.x >= active_wg) return;
    const long long C = P.n_cells;
    const float dr = P.r_max / 32.0f;
    const uint32_t k0 = P.key0, k1 = P.key1;
    const GeoLds geo = stage_geometry(P, s_geo);
    for (int b = lane; b < kBins; b += kWave) bins[b] = 0.0;
    if (lane == 0) reinterpret_cast<uint8_t*>(w_guide16[wv])[kGuide] = kBins - 1;  // the pad entry
    __syncthreads();

    WaveQueue queue = make_queue(n_items, active_wg);
    int item;
    while (next_item(P, queue, item)) {
        if (item < n_chunks) {
            const ChunkInfo ck = load_chunk(P, item);
            const long long hb = (long long)ck.H * kBins;
            reinterpret_cast<v4i*>(cum)[lane] = ((const FCS_AS_GLOBAL v4i*)(G(P.cum) + hb))[lane];
            w_guide16[wv][lane] = ((const FCS_AS_GLOBAL v4i*)(G(P.guide) + (long long)ck.H * kGuide))[lane];
            wave_sync();
            const LayerRec lrec = layer_rec(geo, ck.l);
            const auto g = G(P.grad_cells) + (long long)ck.ev * C;
            double gsum = 0.0;
            for (int i = ck.first + lane; i < ck.first + ck.count; i += kWave) {
                const HitOut h = simulate_hit<true>(geo, lrec, cum, guide, dr, k0, k1, (uint32_t)i,
                                              (uint32_t)ck.l, ck.pin, ck.evg, ck.eta_p, ck.phi_p);
                if (h.cell < 0) continue;
                const double gc = (double)g[h.cell];
                if constexpr (kFluct) {
                    const double x = fluct_factor(h.w4);
                    gsum += gc * x;
                    atomicAdd(&bins[h.bin], gc * (double)(float)((double)ck.ehit * x));
                } else {
                    gsum += gc;
                    atomicAdd(&bins[h.bin], gc * (double)ck.ehit);
                }
            }
#pragma unroll
            for (int d = kWave / 2; d > 0; d >>= 1) gsum += __shfl_xor(gsum, d, kWave);
            if (lane == 0 && gsum != 0.0) gadd(G(P.acc_elayer) + ck.t, gsum);
            wave_sync();
            bool any = false;
            for (int b = lane; b < kBins; b += kWave) {
                const double v = bins[b];
                if (v != 0.0) {
                    gadd(G(P.acc_bins) + hb + b, v);
                    bins[b] = 0.0;
                    any = true;
                }
            }
            if (any) G(P.hist_mark)[ck.H] = 1;  // the weight pass reads this histogram
            wave_sync();
        } else {
            int s0, h0, hcount;
            wave_tile_owners(P, ctr, item - n_chunks, owners, s0, h0, hcount);
            for (int k = lane; k < hcount; k += kWave) {
                const SmallHit sh = small_hit(P, s0 + owners[k], h0 + k);
                const HitOut h = simulate_hit<false>(geo, layer_rec(geo, sh.l),
                                              G(P.cum) + (long long)sh.H * kBins,
                                              G(P.guide) + (long long)sh.H * kGuide, dr, k0, k1,
                                              (uint32_t)sh.i, (uint32_t)sh.l, sh.pin, sh.evg,
                                              sh.eta_p, sh.phi_p);
                if (h.cell < 0) continue;
                const double gc = (double)G(P.grad_cells)[(long long)sh.ev * C + h.cell];
                const double x = kFluct ? fluct_factor(h.w4) : 1.0;
                const float e_hit = kFluct ? (float)((double)sh.ehit * x) : sh.ehit;
                gadd(G(P.acc_elayer) + sh.t, gc * x);
                gadd(G(P.acc_bins) + (long long)sh.H * kBins + h.bin, gc * (double)e_hit);
                G(P.hist_mark)[sh.H] = 1;
            }
            wave_sync();
            // the owner list borrowed the bin sums: zero them again
            for (int b = lane; b < kBins; b += kWave) bins[b] = 0.0;
            wave_sync();
        }
    }
}

// dL/dE_layer = (sum of g, times the hits' energy factors in the fluctuation
// variant, over the task's in-acceptance hits) / n.  The
// accumulator is cleared once read, so the next call starts from zero.
__global__ void k_adj_elayer(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    // asynchronous adjoint calls fold their error bits (all set by now)
    if (t == 0 && P.fold_acc) fold_async(P, P.fold_acc, false, 0);
    if (t >= P.n_tasks) return;
    const int n = G(P.task_n)[t];
    const double a = G(P.acc_elayer)[t];
    if (G(P.grad_elayer)) G(P.grad_elayer)[t] = n > 0 ? (float)(a / (double)n) : 0.0f;
    if (a != 0.0) G(P.acc_elayer)[t] = 0.0;
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// dL/dw_b = A_b / w_b - S / W per histogram, one wave per histogram (four
// bins a lane).  Histograms no task of the call drew from have A = 0 and a
// zero gradient; the others are read, and their sums and mark cleared.
__global__ __launch_bounds__(kBlock) void k_adj_weights(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const int lane = lane_id();
    const long long waves = (long long)gridDim.x * kWavesPerBlock;
    const auto gw = (FCS_AS_GLOBAL v4f*)G(P.grad_weights);
    const auto wv = (const FCS_AS_GLOBAL v4f*)G(P.weights);
    const auto av = (FCS_AS_GLOBAL v2d*)G(P.acc_bins);
    for (long long H = (long long)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; H < P.n_hist;
         H += waves) {
        const long long i = H * (kBins / 4) + lane;  // this lane's four bins
        if (!G(P.hist_mark)[H]) {
            if (gw) gw[i] = v4f{0.f, 0.f, 0.f, 0.f};
            continue;
        }
        const v4f w4 = wv[i];
        const v2d a01 = av[2 * i], a23 = av[2 * i + 1];
        const double W = wave_sum_d(((double)w4.x + (double)w4.y) + ((double)w4.z + (double)w4.w));
        const double S = wave_sum_d((a01.x + a01.y) + (a23.x + a23.y));
        const double q = S / W;
        if (gw) {
            v4f r;
            r.x = (float)((w4.x > 0.f ? a01.x / (double)w4.x : 0.0) - q);
            r.y = (float)((w4.y > 0.f ? a01.y / (double)w4.y : 0.0) - q);
            r.z = (float)((w4.z > 0.f ? a23.x / (double)w4.z : 0.0) - q);
            r.w = (float)((w4.w > 0.f ? a23.y / (double)w4.w : 0.0) - q);
            gw[i] = r;
        }
        av[2 * i] = v2d{0.0, 0.0};
        av[2 * i + 1] = v2d{0.0, 0.0};
        if (lane == 0) G(P.hist_mark)[H] = 0;
    }
}

}  // namespace fcsk
