// Kernels of the batched hit simulation on gfx950 (wave64).
//
// Pipeline of one batch (all launches read one device-resident Params block,
// so the sequence can be captured once in a hipGraph and replayed):
//   k_setup        per (particle, layer): parametrization set, Dirichlet layer
//                  energy, Poisson hit count, Ehit           (Listing 1)
//   k_scan_reduce / k_scan_top / k_scan_write
//                  scans of the task hit counts -> work queue: chunks of
//                  large tasks, packed tiles of small tasks
//   k_hits         persistent: pulls work items from a ticket counter; per
//                  hit Philox draw, inverse-CDF bin, placement, cell lookup,
//                  deposit (sim_a of the CUDA Implementation section)
//   k_seg_count / scan / k_seg_write
//                  ordered gather of the hit cells as (cell_id, E) and
//                  sparse reset of the accumulator (sim_ct and clean)
#pragma once

#include "fcs_math.hpp"

namespace fcsk {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kBins = 256;
constexpr int kHashSlots = 2048;          // LDS cell accumulator of one chunk
constexpr int kHashProbes = 16;
constexpr uint32_t kEmpty = 0xffffffffu;
constexpr int kTileMax = 4096;            // max hits of one packed tile
constexpr int kScanItems = 8;             // items per thread in scans
constexpr int kScanBlock = kBlock * kScanItems;

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
    int32_t ticket;
    int32_t error;        // bit set, see kErr*
    int32_t need_chunks;  // chunk entries required when over capacity
    int32_t pad;
};

enum : int32_t {
    kErrPdg = 1,          // unknown particle type
    kErrParticle = 2,     // non-finite / non-positive inputs
    kErrOffsets = 4,      // malformed event offsets
    kErrTooManyHits = 8,  // more than 2^31-1 hits in one batch
    kErrChunkCap = 16,    // chunk list capacity exceeded (internal retry)
};

struct Params {
    // geometry
    long long n_cells;
    int32_t n_layers, n_regions;
    int32_t n_blk;  // accumulator flag blocks (64 cells) per event
    int32_t n_seg;  // compaction segments (64 flag blocks) per event
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
    int32_t chunk_hits, big_thr, tile_hits;
    int32_t want_hits;
    int32_t clean_cells;  // reset the accumulator while compacting
    int32_t chunk_cap;
    int32_t n_scan_blocks;
    int32_t n_seg_blocks;
    // workspace
    int32_t* task_n;
    float* task_ehit;
    int32_t* part_ev;
    uint32_t* part_p;
    int32_t* part_set;
    int32_t* blk_sums;   // [n_scan_blocks * 4]
    int32_t* blk_offs;   // [n_scan_blocks * 4]
    int32_t* task_hoff;  // [n_tasks] when want_hits
    int4* chunks;        // [chunk_cap] (task key, first hit, count, -)
    int32_t* small_key;  // [n_tasks]
    int32_t* small_off;  // [n_tasks]
    int32_t* tile_first; // [n_tasks + 1]
    float* cells;        // [n_events * n_cells] accumulator
    uint8_t* flags;      // [n_events * n_blk]
    int32_t* seg_cnt;    // [n_events * n_seg]
    int32_t* seg_off;    // [n_events * n_seg]
    int32_t* seg_blk;    // [n_seg_blocks]
    Counters* ctr;
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
    float* grad_elayer;
    float* grad_weights;
    long long n_hist;
};

// ------------------------------------------------------------ utilities ---
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

__device__ __forceinline__ int block_excl_scan1(int v, int& total)
{
    __shared__ int wsum1[kBlock / kWave];
    const int wave = threadIdx.x / kWave;
    const int inc = wave_incl_scan(v);
    if (lane_id() == kWave - 1) wsum1[wave] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        const int s = wsum1[w];
        if (w < wave) off += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return inc - v + off;
}

__device__ __forceinline__ long long block_sum_ll(long long v)
{
    __shared__ long long red[kBlock / kWave];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    if (lane_id() == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    long long t = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) t += red[w];
    __syncthreads();
    return t;
}


__device__ __forceinline__ double block_sum_ll_d(double v)
{
    __shared__ double redd[kBlock / kWave];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    if (lane_id() == 0) redd[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) t += redd[w];
    __syncthreads();
    return t;
}

// inclusive max-scan of the tile owner marks, T / 256 consecutive per thread
__device__ __forceinline__ void owner_max_scan(uint16_t* s_owner, int* s_wmax, int T)
{
    const int tid = threadIdx.x;
    const int per = T / kBlock;
    int m = 0;
    for (int k = 0; k < per; ++k) {
        const int v = s_owner[tid * per + k];
        m = v > m ? v : m;
    }
    int wm = m;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int o = __shfl_up(wm, d, kWave);
        if (lane_id() >= d) wm = o > wm ? o : wm;
    }
    int excl = __shfl_up(wm, 1, kWave);
    if (lane_id() == 0) excl = 0;
    if (lane_id() == kWave - 1) s_wmax[tid / kWave] = wm;
    __syncthreads();
    for (int w = 0; w < tid / kWave; ++w) excl = s_wmax[w] > excl ? s_wmax[w] : excl;
    int run = excl;
    for (int k = 0; k < per; ++k) {
        const int v = s_owner[tid * per + k];
        run = v > run ? v : run;
        s_owner[tid * per + k] = (uint16_t)run;
    }
    __syncthreads();
}

// ---------------------------------------------------- set selection (a1) ---
__device__ __forceinline__ int select_set(const Params& P, int pdg, float e, float eta)
{
    const int apdg = pdg < 0 ? -pdg : pdg;
    const int t = apdg == 11 ? 0 : apdg == 22 ? 1 : apdg == 211 ? 2 : -1;
    if (t < 0) return -1;
    int ie = 0;
    for (int k = 1; k < P.n_ebins; ++k) ie += (e >= P.e_edges[k]) ? 1 : 0;
    const float ae = fabsf(eta);
    int ih = 0;
    for (int k = 1; k < P.n_etabins; ++k) ih += (ae >= P.eta_edges[k]) ? 1 : 0;
    return (t * P.n_ebins + ie) * P.n_etabins + ih;
}

// largest e with ev_off[e] <= gp
__device__ __forceinline__ int find_event(const long long* ev_off, long long n_events, long long gp)
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
    float* p = P.cells;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

__global__ void k_reset_counters(const Params* __restrict__ Pp)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        Counters* c = Pp->ctr;
        c->hits_total = 0;
        c->hits_out = 0;
        c->nnz_total = 0;
        c->n_chunks = 0;
        c->n_small_hits = 0;
        c->n_small_tasks = 0;
        c->n_tiles = 0;
        c->ticket = 0;
        c->error = 0;
        c->need_chunks = 0;
    }
}

// ---------------------------------------------- parametrization tables ---
// cumulative FP32 table per histogram: FP64 running sum over the FP64 total,
// last entry forced to 1
__global__ void k_build_cum(const float* __restrict__ w, float* __restrict__ cum, long long n_hist)
{
    const long long h = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n_hist) return;
    const float* wh = w + h * kBins;
    double tot = 0.0;
    for (int b = 0; b < kBins; ++b) tot = tot + (double)wh[b];
    double acc = 0.0;
    for (int b = 0; b < kBins; ++b) {
        acc = acc + (double)wh[b];
        cum[h * kBins + b] = (float)(acc / tot);
    }
    cum[h * kBins + kBins - 1] = 1.0f;
}

// guide table: g[j] = first bin with cum > j/256, so a draw u with
// floor(256 u) = j lies in bins [g[j], g[j+1]] (g[256] := 255)
__global__ void k_build_guide(const float* __restrict__ cum, uint8_t* __restrict__ guide,
                              long long n_hist)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_hist * kBins) return;
    const long long h = i / kBins;
    const int j = (int)(i - h * kBins);
    const float thr = (float)j * 0x1p-8f;
    const float* c = cum + h * kBins;
    int lo = 0, hi = kBins - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (c[mid] > thr) hi = mid;
        else lo = mid + 1;
    }
    guide[i] = (uint8_t)lo;
}

// ------------------------------------------------- input validation ---
__global__ void k_validate(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int err = 0;
    if (i < P.n_particles) {
        const Particle pt = P.particles[i];
        const int a = pt.pdg < 0 ? -pt.pdg : pt.pdg;
        if (a != 11 && a != 22 && a != 211) err |= kErrPdg;
        if (!(pt.e > 0.0f) || !isfinite(pt.e) || !isfinite(pt.eta) || !isfinite(pt.phi) ||
            fabsf(pt.phi) > 3.2f)
            err |= kErrParticle;
    }
    if (i < P.n_events) {
        if (P.ev_off[i] > P.ev_off[i + 1]) err |= kErrOffsets;
    }
    if (i == 0) {
        if (P.ev_off[0] != P.part_base || P.ev_off[P.n_events] != P.part_base + P.n_particles)
            err |= kErrOffsets;
    }
    if (err) atomicOr(&P.ctr->error, err);
}

// ------------------------------------------- per-task setup (a1 - a3) ---
// One thread per (particle, layer); the particles of a block share their
// Gamma draws through LDS for the Dirichlet normalization.
__global__ __launch_bounds__(kBlock) void k_setup(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    __shared__ double g_s[kBlock];
    const int L = P.n_layers;
    const int ppb = kBlock / L;
    const int tid = threadIdx.x;
    const int lp = tid / L;
    const int l = tid - lp * L;
    const long long gp = (long long)blockIdx.x * ppb + lp;
    const bool active = lp < ppb && gp < P.n_particles;
    Particle pt = {0, 0.f, 0.f, 0.f};
    int set = -1, ev = 0;
    uint32_t pin = 0, evg = 0;
    double g = 0.0;
    if (active) {
        pt = P.particles[gp];
        ev = find_event(P.ev_off, P.n_events, P.part_base + gp);
        pin = (uint32_t)(P.part_base + gp - P.ev_off[ev]);
        evg = (uint32_t)(P.ev_base + (unsigned long long)ev);
        set = select_set(P, pt.pdg, pt.e, pt.eta);
        if (set >= 0) {
            const int t = set / (P.n_ebins * P.n_etabins);
            g = gamma_draw((double)P.alpha[t * L + l], P.key0, P.key1, (uint32_t)l, pin, evg);
        }
    }
    g_s[tid] = g;
    __syncthreads();
    if (!active) return;
    int n = 0;
    float ehit = 0.0f;
    double el = 0.0;
    const long long t = gp * L + l;
    if (set >= 0) {
        double sum = 0.0;
        for (int k = 0; k < L; ++k) sum = sum + g_s[lp * L + k];
        el = (double)pt.e * (g / sum);
        if (el >= P.min_e && el > 0.0) {
            const double mu = el / (double)P.scale;
            long long k = poisson_draw(mu, P.key0, P.key1, (uint32_t)l, pin, evg);
            if (k < 1) k = 1;
            if (k > P.cap) k = P.cap;
            n = (int)k;
        }
        const double e_used = P.elayer_override ? (double)P.elayer_override[t] : el;
        ehit = n > 0 ? (float)(e_used / (double)n) : 0.0f;
    }
    P.task_n[t] = n;
    P.task_ehit[t] = ehit;
    if (P.out_elayer) P.out_elayer[t] = (float)el;
    if (P.out_counts) P.out_counts[t] = n;
    if (l == 0) {
        P.part_ev[gp] = ev;
        P.part_p[gp] = pin;
        P.part_set[gp] = set;
    }
}

// ----------------------------------------- task scans -> work queue (a11) ---
// per task: x = hits, y = chunks of a large task, z = hits of a small task,
// w = 1 for a small task with hits
__device__ __forceinline__ int4 task_terms(const Params& P, int n)
{
    const bool big = n >= P.big_thr;
    return make_int4(n, big ? (n + P.chunk_hits - 1) / P.chunk_hits : 0, (!big && n > 0) ? n : 0,
                     (!big && n > 0) ? 1 : 0);
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const long long base = (long long)blockIdx.x * kScanBlock + (long long)threadIdx.x * kScanItems;
    int4 s = make_int4(0, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const long long t = base + k;
        if (t < P.n_tasks) s = add4(s, task_terms(P, P.task_n[t]));
    }
    int4 tot;
    (void)block_excl_scan4(s, tot);
    if (threadIdx.x == 0) reinterpret_cast<int4*>(P.blk_sums)[blockIdx.x] = tot;
}

// one block: exclusive scan of the block sums; totals into the counters
__global__ __launch_bounds__(1024) void k_scan_top(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    __shared__ long long carry_s[4];
    __shared__ long long part_s[1024 / kWave][4];
    const int tid = threadIdx.x;
    if (tid < 4) carry_s[tid] = 0;
    __syncthreads();
    const int nb = P.n_scan_blocks;
    const int4* in = reinterpret_cast<const int4*>(P.blk_sums);
    int4* out = reinterpret_cast<int4*>(P.blk_offs);
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int b = b0 + tid;
        const int4 v = b < nb ? in[b] : make_int4(0, 0, 0, 0);
        long long x[4] = {v.x, v.y, v.z, v.w};
        long long inc[4];
        for (int c = 0; c < 4; ++c) inc[c] = wave_incl_scan<long long>(x[c]);
        const int wave = tid / kWave;
        if (lane_id() == kWave - 1)
            for (int c = 0; c < 4; ++c) part_s[wave][c] = inc[c];
        __syncthreads();
        long long off[4] = {0, 0, 0, 0}, tot[4] = {0, 0, 0, 0};
        for (int w = 0; w < 1024 / kWave; ++w)
            for (int c = 0; c < 4; ++c) {
                if (w < wave) off[c] += part_s[w][c];
                tot[c] += part_s[w][c];
            }
        if (b < nb) {
            int4 o;
            o.x = (int)(carry_s[0] + off[0] + inc[0] - x[0]);
            o.y = (int)(carry_s[1] + off[1] + inc[1] - x[1]);
            o.z = (int)(carry_s[2] + off[2] + inc[2] - x[2]);
            o.w = (int)(carry_s[3] + off[3] + inc[3] - x[3]);
            out[b] = o;
        }
        __syncthreads();
        if (tid < 4) carry_s[tid] += tot[tid];
        __syncthreads();
    }
    if (tid == 0) {
        Counters* c = P.ctr;
        c->hits_total = carry_s[0];
        int err = 0;
        if (carry_s[0] > 2147483647LL) err |= kErrTooManyHits;
        if (carry_s[1] > P.chunk_cap) {
            err |= kErrChunkCap;
            c->need_chunks = (int)(carry_s[1] < 2147483647LL ? carry_s[1] : 2147483647LL);
        }
        c->n_chunks = err ? 0 : (int)carry_s[1];
        c->n_small_hits = err ? 0 : (int)carry_s[2];
        c->n_small_tasks = err ? 0 : (int)carry_s[3];
        c->n_tiles = err ? 0 : (int)((carry_s[2] + P.tile_hits - 1) / P.tile_hits);
        c->ticket = 0;
        if (err) atomicOr(&c->error, err);
        if (P.out_task_hoff && !err) P.out_task_hoff[P.n_tasks] = P.hit_base + carry_s[0];
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_write(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    if (P.ctr->error & (kErrTooManyHits | kErrChunkCap)) return;
    const long long base = (long long)blockIdx.x * kScanBlock + (long long)threadIdx.x * kScanItems;
    int nv[kScanItems];
    int4 s = make_int4(0, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const long long t = base + k;
        nv[k] = t < P.n_tasks ? P.task_n[t] : 0;
        s = add4(s, task_terms(P, nv[k]));
    }
    int4 tot;
    int4 run = add4(block_excl_scan4(s, tot), reinterpret_cast<const int4*>(P.blk_offs)[blockIdx.x]);
    const int L = P.n_layers;
    for (int k = 0; k < kScanItems; ++k) {
        const long long t = base + k;
        if (t >= P.n_tasks) break;
        const int n = nv[k];
        const int4 d = task_terms(P, n);
        if (P.want_hits) P.task_hoff[t] = run.x;
        if (P.out_task_hoff) P.out_task_hoff[t] = P.hit_base + run.x;
        const long long gp = t / L;
        const int key = (int)(gp * 64 + (t - gp * L));
        for (int c = 0; c < d.y; ++c) {
            const int first = c * P.chunk_hits;
            const int cnt = min(P.chunk_hits, n - first);
            P.chunks[run.y + c] = make_int4(key, first, cnt, 0);
        }
        if (d.w) {
            P.small_key[run.w] = key;
            P.small_off[run.w] = run.z;
            const int T = P.tile_hits;
            const int q = (run.z + T - 1) / T;
            if ((long long)q * T < (long long)run.z + n) P.tile_first[q] = run.w;
        }
        run = add4(run, d);
    }
}

// ------------------------------------------------------ the hit (a4 - a7) ---
struct Region {
    float eta_lo, inv_deta, phi_lo, inv_dphi;
    int neta, nphi, off;
};

// region grid lookup: -1 outside [eta_lo(first), eta_hi(last))
__device__ __forceinline__ int lookup_cell(const Params& P, int l, float eta, float phi)
{
    const int R = P.n_regions;
    const int base = l * R;
    if (!(eta >= P.reg_eta_lo[base]) || !(eta < P.reg_eta_hi[base + R - 1])) return -1;
    int k = 0;
    for (int j = 1; j < R; ++j) k += (eta >= P.reg_eta_lo[base + j]) ? 1 : 0;
    const int r = base + k;
    const int ne = P.reg_neta[r], np = P.reg_nphi[r];
    int ie = (int)floorf((eta - P.reg_eta_lo[r]) * P.reg_inv_deta[r]);
    int ip = (int)floorf((phi - P.reg_phi_lo[r]) * P.reg_inv_dphi[r]);
    ie = min(max(ie, 0), ne - 1);
    ip = min(max(ip, 0), np - 1);
    return P.reg_offset[r] + ie * np + ip;
}

// first bin with cum > u; the guide narrows the search to [g[j], g[j+1]]
template <typename CumT, typename GuideT>
__device__ __forceinline__ int find_bin(CumT cum, GuideT guide, uint32_t x0, float u)
{
    const int j = (int)(x0 >> 24);
    int lo = guide[j];
    int hi = j < kBins - 1 ? (int)guide[j + 1] : kBins - 1;
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
};

template <typename CumT, typename GuideT>
__device__ __forceinline__ HitOut simulate_hit(const Params& P, CumT cum, GuideT guide, uint32_t i,
                                               uint32_t l, uint32_t pin, uint32_t evg, float eta_p,
                                               float phi_p, float inv_r)
{
    const U4 x = philox4x32_10(i, l | (kTagHit << 8), pin, evg, P.key0, P.key1);
    const float u0 = unit24(x.x), u1 = unit24(x.y), u2 = unit24(x.z);
    HitOut h;
    h.bin = find_bin(cum, guide, x.x, u0);
    const int ir = h.bin >> 3, ia = h.bin & 7;
    const float dr = P.r_max / 32.0f;
    const float r = (float)ir * dr + u1 * dr;
    float c, s;
    sincos_bin(ia, u2, c, s);
    const float deta = (r * c) * inv_r;
    const float dphi = (r * s) * inv_r;
    const float eta = eta_p + deta;
    float phi = phi_p + dphi;
    const float pi_f = 3.14159265358979323846f;
    const float two_pi_f = 6.28318530717958647692f;
    if (phi >= pi_f) phi = phi - two_pi_f;
    else if (phi < -pi_f) phi = phi + two_pi_f;
    h.eta = eta;
    h.phi = phi;
    h.cell = lookup_cell(P, (int)l, eta, phi);
    return h;
}

__device__ __forceinline__ void write_hit(const Params& P, long long pos, const HitOut& h, float e)
{
    pos += P.hit_base;
    if (pos < P.hit_cap) {
        P.hit_eta[pos] = h.eta;
        P.hit_phi[pos] = h.phi;
        P.hit_e[pos] = e;
        P.hit_cell[pos] = h.cell;
    }
}

// ------------------------------------------------- persistent hit kernel ---
// Work items: [0, n_chunks) chunks of large tasks, then packed tiles of small
// tasks.  A chunk belongs to one (particle, layer): its histogram and guide
// sit in LDS and its hits are counted per cell in an LDS hash table, flushed
// once as count * Ehit (one rounding per cell and chunk).  Tile hits add
// their energy to the event's cell with one device atomic each.
__global__ __launch_bounds__(kBlock) void k_hits(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    __shared__ uint32_t h_key[kHashSlots];
    __shared__ uint32_t h_cnt[kHashSlots];
    __shared__ float s_cum[kBins];
    __shared__ uint8_t s_guide[kBins];
    __shared__ uint16_t s_owner[kTileMax];
    __shared__ int s_wmax[kBlock / kWave];
    __shared__ int s_item;

    const int tid = threadIdx.x;
    const Counters* ctr = P.ctr;
    if (ctr->error & (kErrTooManyHits | kErrChunkCap)) return;
    const int n_chunks = ctr->n_chunks;
    const int n_items = n_chunks + ctr->n_tiles;
    const int L = P.n_layers;
    const long long C = P.n_cells;
    long long n_out = 0;

    for (int s = tid; s < kHashSlots; s += kBlock) {
        h_key[s] = kEmpty;
        h_cnt[s] = 0;
    }

    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = atomicAdd(&P.ctr->ticket, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= n_items) break;

        if (item < n_chunks) {
            // ------------------------------------------- chunk of a large task
            const int4 ck = P.chunks[item];
            const long long gp = ck.x >> 6;
            const int l = ck.x & 63;
            const long long t = gp * L + l;
            const float ehit = P.task_ehit[t];
            const int ev = P.part_ev[gp];
            const uint32_t pin = P.part_p[gp];
            const uint32_t evg = (uint32_t)(P.ev_base + (unsigned long long)ev);
            const long long H = (long long)P.part_set[gp] * L + l;
            const Particle pt = P.particles[gp];
            const float inv_r = P.layer_inv_r[l];
            s_cum[tid] = P.cum[H * kBins + tid];
            s_guide[tid] = P.guide[H * kBins + tid];
            __syncthreads();
            float* cells_e = P.cells + (long long)ev * C;
            const long long hbase = P.want_hits ? (long long)P.task_hoff[t] : 0;
            for (int i = ck.y + tid; i < ck.y + ck.z; i += kBlock) {
                const HitOut h = simulate_hit(P, s_cum, s_guide, (uint32_t)i, (uint32_t)l, pin, evg,
                                              pt.eta, pt.phi, inv_r);
                if (P.want_hits) write_hit(P, hbase + i, h, ehit);
                if (h.cell < 0) {
                    ++n_out;
                    continue;
                }
                const uint32_t key = (uint32_t)h.cell;
                uint32_t slot = (key * 2654435761u) >> (32 - 11);
                bool done = false;
                for (int pr = 0; pr < kHashProbes; ++pr) {
                    const uint32_t old = atomicCAS(&h_key[slot], kEmpty, key);
                    if (old == kEmpty || old == key) {
                        atomicAdd(&h_cnt[slot], 1u);
                        done = true;
                        break;
                    }
                    slot = (slot + 1) & (kHashSlots - 1);
                }
                if (!done) {
                    unsafeAtomicAdd(cells_e + h.cell, ehit);
                    P.flags[(long long)ev * P.n_blk + (h.cell >> 6)] = 1;
                }
            }
            __syncthreads();
            for (int s = tid; s < kHashSlots; s += kBlock) {
                const uint32_t key = h_key[s];
                if (key != kEmpty) {
                    unsafeAtomicAdd(cells_e + key, (float)h_cnt[s] * ehit);
                    P.flags[(long long)ev * P.n_blk + (key >> 6)] = 1;
                    h_key[s] = kEmpty;
                    h_cnt[s] = 0;
                }
            }
        } else {
            // ------------------------------------------ tile of small tasks
            const int q = item - n_chunks;
            const int T = P.tile_hits;
            const int h0 = q * T;
            const int hcount = min(T, ctr->n_small_hits - h0);
            const int s0 = P.tile_first[q];
            const int s1 = (q + 1 < ctr->n_tiles) ? P.tile_first[q + 1] : ctr->n_small_tasks - 1;
            for (int k = tid; k < T; k += kBlock) s_owner[k] = 0;
            __syncthreads();
            for (int j = s0 + tid; j <= s1; j += kBlock) {
                int st = P.small_off[j] - h0;
                st = st < 0 ? 0 : st;
                if (st < T) s_owner[st] = (uint16_t)(j - s0);
            }
            __syncthreads();
            owner_max_scan(s_owner, s_wmax, T);
            for (int k = tid; k < hcount; k += kBlock) {
                const int j = s0 + s_owner[k];
                const int key = P.small_key[j];
                const long long gp = key >> 6;
                const int l = key & 63;
                const long long t = gp * L + l;
                const int i = h0 + k - P.small_off[j];
                const float ehit = P.task_ehit[t];
                const int ev = P.part_ev[gp];
                const uint32_t evg = (uint32_t)(P.ev_base + (unsigned long long)ev);
                const long long H = (long long)P.part_set[gp] * L + l;
                const Particle pt = P.particles[gp];
                const HitOut h = simulate_hit(P, P.cum + H * kBins, P.guide + H * kBins, (uint32_t)i,
                                              (uint32_t)l, P.part_p[gp], evg, pt.eta, pt.phi,
                                              P.layer_inv_r[l]);
                if (P.want_hits) write_hit(P, (long long)P.task_hoff[t] + i, h, ehit);
                if (h.cell < 0) {
                    ++n_out;
                    continue;
                }
                unsafeAtomicAdd(P.cells + (long long)ev * C + h.cell, ehit);
                P.flags[(long long)ev * P.n_blk + (h.cell >> 6)] = 1;
            }
        }
    }
    const long long tot = block_sum_ll(n_out);
    if (tid == 0 && tot)
        atomicAdd(reinterpret_cast<unsigned long long*>(&P.ctr->hits_out), (unsigned long long)tot);
}

// ------------------------------------------ ordered compaction (a10) ---
// One wave per segment of 64 flag blocks (4096 cells) of one event.  Only
// flagged blocks are read; ballots give each lane its output slot, so the
// output is in ascending dense cell index per event.
__global__ __launch_bounds__(kBlock) void k_seg_count(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const long long gw = (long long)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (gw >= P.n_events * P.n_seg) return;
    const long long e = gw / P.n_seg;
    const int seg = (int)(gw - e * P.n_seg);
    const int lane = lane_id();
    const int fb = seg * 64 + lane;
    const bool flagged = fb < P.n_blk && P.flags[e * P.n_blk + fb] != 0;
    unsigned long long mask = __ballot(flagged);
    const float* cells = P.cells + e * P.n_cells;
    int cnt = 0;
    while (mask) {
        const int b = __ffsll((long long)mask) - 1;
        mask &= mask - 1;
        const long long cell = (long long)(seg * 64 + b) * 64 + lane;
        const float v = cell < P.n_cells ? cells[cell] : 0.0f;
        cnt += __popcll(__ballot(v != 0.0f));
    }
    if (lane == 0) P.seg_cnt[gw] = cnt;
}

__global__ __launch_bounds__(kBlock) void k_seg_reduce(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const long long n = P.n_events * P.n_seg;
    const long long base = (long long)blockIdx.x * kScanBlock + (long long)threadIdx.x * kScanItems;
    int s = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += P.seg_cnt[base + k];
    int tot;
    (void)block_excl_scan1(s, tot);
    if (threadIdx.x == 0) P.seg_blk[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_seg_top(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    __shared__ long long carry;
    __shared__ long long part[1024 / kWave];
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    const int nb = P.n_seg_blocks;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int b = b0 + tid;
        const long long v = b < nb ? P.seg_blk[b] : 0;
        const long long inc = wave_incl_scan<long long>(v);
        if (lane_id() == kWave - 1) part[tid / kWave] = inc;
        __syncthreads();
        long long off = 0, tot = 0;
        for (int w = 0; w < 1024 / kWave; ++w) {
            if (w < tid / kWave) off += part[w];
            tot += part[w];
        }
        if (b < nb) P.seg_blk[b] = (int)(carry + off + inc - v);
        __syncthreads();
        if (tid == 0) carry += tot;
        __syncthreads();
    }
    if (tid == 0) {
        P.ctr->nnz_total = carry;
        if (P.out_ev_off) P.out_ev_off[P.n_events] = P.out_base + carry;
    }
}

__global__ __launch_bounds__(kBlock) void k_seg_apply(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const long long n = P.n_events * P.n_seg;
    const long long base = (long long)blockIdx.x * kScanBlock + (long long)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? P.seg_cnt[base + k] : 0;
        s += v[k];
    }
    int tot;
    int run = block_excl_scan1(s, tot) + P.seg_blk[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) P.seg_off[base + k] = run;
        run += v[k];
    }
}

__global__ __launch_bounds__(kBlock) void k_seg_write(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const long long gw = (long long)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (gw >= P.n_events * P.n_seg) return;
    const long long e = gw / P.n_seg;
    const int seg = (int)(gw - e * P.n_seg);
    const int lane = lane_id();
    const int fb = seg * 64 + lane;
    const bool flagged = fb < P.n_blk && P.flags[e * P.n_blk + fb] != 0;
    unsigned long long mask = __ballot(flagged);
    float* cells = P.cells + e * P.n_cells;
    long long pos = P.out_base + P.seg_off[gw];
    if (seg == 0 && lane == 0 && P.out_ev_off) P.out_ev_off[e] = pos;
    const unsigned long long below = (1ull << lane) - 1ull;
    while (mask) {
        const int b = __ffsll((long long)mask) - 1;
        mask &= mask - 1;
        const long long cell = (long long)(seg * 64 + b) * 64 + lane;
        const bool in = cell < P.n_cells;
        const float v = in ? cells[cell] : 0.0f;
        const unsigned long long nz = __ballot(v != 0.0f);
        if (v != 0.0f) {
            const long long o = pos + __popcll(nz & below);
            if (o < P.out_cap) {
                P.out_ids[o] = P.cell_id[cell];
                P.out_e[o] = v;
            }
        }
        if (P.clean_cells && in) cells[cell] = 0.0f;
        pos += __popcll(nz);
    }
    if (flagged) P.flags[e * P.n_blk + fb] = 0;
}


// ------------------------------------------------------ adjoint (a12) ---
// Same work items as k_hits.  Each hit's bin and cell are recomputed from its
// Philox counter; g = dL/dE_cell is gathered at the cell and accumulated in
// FP64 per task (sum of g) and per histogram bin (sum of g * Ehit).  A chunk
// of a large task keeps its 256 bin sums in LDS and flushes them once.
__global__ __launch_bounds__(kBlock) void k_adjoint(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    __shared__ float s_cum[kBins];
    __shared__ uint8_t s_guide[kBins];
    __shared__ double s_bin[kBins];
    __shared__ uint16_t s_owner[kTileMax];
    __shared__ int s_wmax[kBlock / kWave];
    __shared__ int s_item;

    const int tid = threadIdx.x;
    const Counters* ctr = P.ctr;
    if (ctr->error & (kErrTooManyHits | kErrChunkCap)) return;
    const int n_chunks = ctr->n_chunks;
    const int n_items = n_chunks + ctr->n_tiles;
    const int L = P.n_layers;
    const long long C = P.n_cells;
    s_bin[tid] = 0.0;

    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = atomicAdd(&P.ctr->ticket, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= n_items) break;
        if (item < n_chunks) {
            const int4 ck = P.chunks[item];
            const long long gp = ck.x >> 6;
            const int l = ck.x & 63;
            const long long t = gp * L + l;
            const float ehit = P.task_ehit[t];
            const int ev = P.part_ev[gp];
            const uint32_t pin = P.part_p[gp];
            const uint32_t evg = (uint32_t)(P.ev_base + (unsigned long long)ev);
            const long long H = (long long)P.part_set[gp] * L + l;
            const Particle pt = P.particles[gp];
            const float inv_r = P.layer_inv_r[l];
            s_cum[tid] = P.cum[H * kBins + tid];
            s_guide[tid] = P.guide[H * kBins + tid];
            __syncthreads();
            const float* g = P.grad_cells + (long long)ev * C;
            double gsum = 0.0;
            for (int i = ck.y + tid; i < ck.y + ck.z; i += kBlock) {
                const HitOut h = simulate_hit(P, s_cum, s_guide, (uint32_t)i, (uint32_t)l, pin, evg,
                                              pt.eta, pt.phi, inv_r);
                if (h.cell < 0) continue;
                const double gc = (double)g[h.cell];
                gsum += gc;
                atomicAdd(&s_bin[h.bin], gc * (double)ehit);
            }
            gsum = block_sum_ll_d(gsum);
            if (tid == 0 && gsum != 0.0) unsafeAtomicAdd(P.acc_elayer + t, gsum);
            __syncthreads();
            const double v = s_bin[tid];
            if (v != 0.0) {
                unsafeAtomicAdd(P.acc_bins + H * kBins + tid, v);
                s_bin[tid] = 0.0;
            }
        } else {
            const int q = item - n_chunks;
            const int T = P.tile_hits;
            const int h0 = q * T;
            const int hcount = min(T, ctr->n_small_hits - h0);
            const int s0 = P.tile_first[q];
            const int s1 = (q + 1 < ctr->n_tiles) ? P.tile_first[q + 1] : ctr->n_small_tasks - 1;
            for (int k = tid; k < T; k += kBlock) s_owner[k] = 0;
            __syncthreads();
            for (int j = s0 + tid; j <= s1; j += kBlock) {
                int st = P.small_off[j] - h0;
                st = st < 0 ? 0 : st;
                if (st < T) s_owner[st] = (uint16_t)(j - s0);
            }
            __syncthreads();
            owner_max_scan(s_owner, s_wmax, T);
            for (int k = tid; k < hcount; k += kBlock) {
                const int j = s0 + s_owner[k];
                const int key = P.small_key[j];
                const long long gp = key >> 6;
                const int l = key & 63;
                const long long t = gp * L + l;
                const int i = h0 + k - P.small_off[j];
                const float ehit = P.task_ehit[t];
                const int ev = P.part_ev[gp];
                const uint32_t evg = (uint32_t)(P.ev_base + (unsigned long long)ev);
                const long long H = (long long)P.part_set[gp] * L + l;
                const Particle pt = P.particles[gp];
                const HitOut h = simulate_hit(P, P.cum + H * kBins, P.guide + H * kBins, (uint32_t)i,
                                              (uint32_t)l, P.part_p[gp], evg, pt.eta, pt.phi,
                                              P.layer_inv_r[l]);
                if (h.cell < 0) continue;
                const double gc = (double)P.grad_cells[(long long)ev * C + h.cell];
                unsafeAtomicAdd(P.acc_elayer + t, gc);
                unsafeAtomicAdd(P.acc_bins + H * kBins + h.bin, gc * (double)ehit);
            }
        }
    }
}

// dL/dE_layer = (sum of g over the task's in-acceptance hits) / n
__global__ void k_adj_elayer(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P.n_tasks) return;
    const int n = P.task_n[t];
    P.grad_elayer[t] = n > 0 ? (float)(P.acc_elayer[t] / (double)n) : 0.0f;
}

// dL/dw_b = A_b / w_b - S / W per histogram (one block per histogram)
__global__ __launch_bounds__(kBlock) void k_adj_weights(const Params* __restrict__ Pp)
{
    const Params& P = *Pp;
    const long long H = blockIdx.x;
    const int b = threadIdx.x;
    const double w = (double)P.weights[H * kBins + b];
    const double A = P.acc_bins[H * kBins + b];
    const double W = block_sum_ll_d(w);
    const double S = block_sum_ll_d(A);
    const double lr = w > 0.0 ? A / w : 0.0;
    P.grad_weights[H * kBins + b] = (float)(lr - S / W);
}

}  // namespace fcsk
