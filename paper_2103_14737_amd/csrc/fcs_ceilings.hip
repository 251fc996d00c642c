// Measured ceilings of the chip for the kernels of the hit simulation:
// device FP32 atomic adds (the deposit), an HBM copy (the dense cell passes),
// a Philox4x32-10-only VALU kernel with the shader clock it runs at, and the
// cost of a kernel launch (plain stream launches, hipGraph launches, and a
// launch waited for by the host, as the per-event form pays it).
//
// A separate library (libfcs_ceilings.so) used by the benchmark only; it
// shares the Philox generator of the hit kernels so that the VALU ceiling
// times the same instructions.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "fcs_math.hpp"

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    // a 32-bit integer finalizer (Murmur3's fmix32) for pseudo-random indices
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    return x;
}

// One FP32 atomic add of 1 per op into cells[n_cells].  pattern 0: cells
// uniform over the array; pattern 1: "showers", every 64 consecutive ops (one
// wave) around one random centre, at a distance drawn from an exponential of
// mean 8 cells on either side; pattern 2: "rows", the 64 lanes of a wave on
// 64 consecutive cells starting at a random multiple of 64 (the coalesced
// flush of an accumulator window).  kReturning: the instruction returns the old
// value (as the deposits that count new cells use it); else it is issued
// without a return.
template <bool kReturning>
__global__ __launch_bounds__(kThreads) void k_atomic(float* __restrict__ cells, uint32_t n_cells,
                                                     long long n_ops, int pattern, uint32_t seed,
                                                     float* __restrict__ sink)
{
    float acc = 0.0f;
    const long long stride = (long long)gridDim.x * kThreads;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n_ops; i += stride) {
        const uint32_t h = mix32((uint32_t)i * 0x9E3779B9u ^ seed);
        uint32_t idx;
        if (pattern == 0) {
            idx = (uint32_t)(((uint64_t)h * n_cells) >> 32);
        } else if (pattern == 2) {
            const uint32_t rows = n_cells / 64;
            const uint32_t r = (uint32_t)(((uint64_t)mix32((uint32_t)(i >> 6) ^ seed) * rows) >> 32);
            idx = r * 64u + (uint32_t)(i & 63);
        } else {
            const uint32_t c = (uint32_t)(((uint64_t)mix32((uint32_t)(i >> 6) ^ seed ^ 0x5bd1e995u) * n_cells) >> 32);
            const float u = ((float)(h >> 8) + 0.5f) * 0x1p-24f;
            const int d = (int)(-8.0f * __logf(u));
            long long j = (h & 1u) ? (long long)c + d : (long long)c - d;
            j = j < 0 ? 0 : (j >= (long long)n_cells ? (long long)n_cells - 1 : j);
            idx = (uint32_t)j;
        }
        if constexpr (kReturning) {
            acc += __hip_atomic_fetch_add(cells + idx, 1.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            (void)__hip_atomic_fetch_add(cells + idx, 1.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (kReturning && acc < 0.0f) sink[0] = acc;  // keeps the returned values live
}

__global__ __launch_bounds__(kThreads) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                   long long n)
{
    const long long stride = (long long)gridDim.x * kThreads;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// n_draws Philox4x32-10 draws per lane, counters as a hit's (draw, tag,
// lane, workgroup), the words xor-folded into one output per lane.  Thread 0
// of every workgroup records the shader clock counter (s_memtime) and the
// constant 100 MHz counter (s_memrealtime) when it starts and ends.
__global__ __launch_bounds__(kThreads) void k_philox(uint32_t n_draws, uint32_t k0, uint32_t k1,
                                                     uint32_t* __restrict__ out,
                                                     unsigned long long* __restrict__ clocks)
{
    unsigned long long t0 = 0, r0 = 0;
    if (threadIdx.x == 0) {
        t0 = __builtin_amdgcn_s_memtime();
        r0 = __builtin_amdgcn_s_memrealtime();
    }
    uint32_t acc = 0;
    for (uint32_t i = 0; i < n_draws; ++i) {
        const fcsk::U4 x = fcsk::philox4x32_10(i, 3u << 8, threadIdx.x, blockIdx.x, k0, k1);
        acc ^= x.x ^ x.y ^ x.z ^ x.w;
    }
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = acc;
    if (threadIdx.x == 0) {
        const unsigned long long t1 = __builtin_amdgcn_s_memtime();
        const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
        clocks[2 * blockIdx.x] = t1 - t0;
        clocks[2 * blockIdx.x + 1] = r1 - r0;
    }
}

__global__ void k_empty() {}

#define CHK(call)                                                  \
    do {                                                           \
        if ((call) != hipSuccess) {                                \
            (void)hipGetLastError();                               \
            return -1;                                             \
        }                                                          \
    } while (0)

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    ~Timer()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

extern "C" {

// FP32 atomic adds per second: n_ops adds (pattern 0 uniform, 1 showers, 2 rows)
// into n_cells cells, over `reps` launches after one warm-up launch.
int fcs_ceil_atomic(int device, long long n_cells, long long n_ops, int pattern, int returning, int reps,
                    double* ops_per_s)
{
    if (n_cells < 1 || n_cells > (1LL << 31) || n_ops < 1 || reps < 1 || !ops_per_s) return -2;
    CHK(hipSetDevice(device));
    float *cells = nullptr, *sink = nullptr;
    CHK(hipMalloc(&cells, (size_t)n_cells * 4));
    CHK(hipMalloc(&sink, 4));
    CHK(hipMemset(cells, 0, (size_t)n_cells * 4));
    Timer t;
    CHK(hipEventCreate(&t.a));
    CHK(hipEventCreate(&t.b));
    hipDeviceProp_t prop;
    CHK(hipGetDeviceProperties(&prop, device));
    const dim3 grid(prop.multiProcessorCount * 8);
    int rc = 0;
    for (int r = -1; r < reps; ++r) {
        if (r == 0) CHK(hipEventRecord(t.a, nullptr));
        if (returning)
            hipLaunchKernelGGL(k_atomic<true>, grid, dim3(kThreads), 0, nullptr, cells, (uint32_t)n_cells,
                               n_ops, pattern, 0x1234u + (uint32_t)r, sink);
        else
            hipLaunchKernelGGL(k_atomic<false>, grid, dim3(kThreads), 0, nullptr, cells, (uint32_t)n_cells,
                               n_ops, pattern, 0x1234u + (uint32_t)r, sink);
    }
    CHK(hipEventRecord(t.b, nullptr));
    CHK(hipEventSynchronize(t.b));
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, t.a, t.b));
    *ops_per_s = (double)n_ops * reps / (ms * 1e-3);
    if (hipFree(cells) != hipSuccess || hipFree(sink) != hipSuccess) rc = -1;
    return rc;
}

// HBM copy: bytes read + written per second for a device copy of `bytes`.
int fcs_ceil_copy(int device, long long bytes, int reps, double* bytes_per_s)
{
    if (bytes < 16 || reps < 1 || !bytes_per_s) return -2;
    CHK(hipSetDevice(device));
    const long long n = bytes / 16;
    float4 *a = nullptr, *b = nullptr;
    CHK(hipMalloc(&a, (size_t)n * 16));
    CHK(hipMalloc(&b, (size_t)n * 16));
    CHK(hipMemset(a, 0, (size_t)n * 16));
    Timer t;
    CHK(hipEventCreate(&t.a));
    CHK(hipEventCreate(&t.b));
    hipDeviceProp_t prop;
    CHK(hipGetDeviceProperties(&prop, device));
    const dim3 grid(prop.multiProcessorCount * 8);
    for (int r = -1; r < reps; ++r) {
        if (r == 0) CHK(hipEventRecord(t.a, nullptr));
        hipLaunchKernelGGL(k_copy, grid, dim3(kThreads), 0, nullptr, a, b, n);
    }
    CHK(hipEventRecord(t.b, nullptr));
    CHK(hipEventSynchronize(t.b));
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, t.a, t.b));
    *bytes_per_s = 2.0 * (double)n * 16 * reps / (ms * 1e-3);
    CHK(hipFree(a));
    CHK(hipFree(b));
    return 0;
}

// Device-to-host DMA copy into pinned host memory (hipHostMalloc):
// bytes per second for copies of `bytes`, one stream, `reps` copies.
int fcs_ceil_d2h(int device, long long bytes, int reps, double* bytes_per_s)
{
    if (bytes < 1 || reps < 1 || !bytes_per_s) return -2;
    CHK(hipSetDevice(device));
    void *d = nullptr, *h = nullptr;
    CHK(hipMalloc(&d, (size_t)bytes));
    CHK(hipMemset(d, 0, (size_t)bytes));
    CHK(hipHostMalloc(&h, (size_t)bytes, hipHostMallocDefault));
    hipStream_t s = nullptr;
    CHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    Timer t;
    CHK(hipEventCreate(&t.a));
    CHK(hipEventCreate(&t.b));
    CHK(hipMemcpyAsync(h, d, (size_t)bytes, hipMemcpyDeviceToHost, s));
    CHK(hipEventRecord(t.a, s));
    for (int r = 0; r < reps; ++r) CHK(hipMemcpyAsync(h, d, (size_t)bytes, hipMemcpyDeviceToHost, s));
    CHK(hipEventRecord(t.b, s));
    CHK(hipEventSynchronize(t.b));
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, t.a, t.b));
    *bytes_per_s = (double)bytes * reps / (ms * 1e-3);
    CHK(hipStreamDestroy(s));
    CHK(hipFree(d));
    CHK(hipHostFree(h));
    return 0;
}

// Philox4x32-10 draws per second over `workgroups` x 256 lanes of n_draws
// each, and the mean shader clock of the workgroups while they ran (their
// s_memtime cycles over s_memrealtime time).
int fcs_ceil_philox(int device, int workgroups, int n_draws, double* draws_per_s, double* clock_hz)
{
    if (workgroups < 1 || n_draws < 1 || !draws_per_s || !clock_hz) return -2;
    CHK(hipSetDevice(device));
    uint32_t* out = nullptr;
    unsigned long long* clk = nullptr;
    CHK(hipMalloc(&out, (size_t)workgroups * kThreads * 4));
    CHK(hipMalloc(&clk, (size_t)workgroups * 16));
    Timer t;
    CHK(hipEventCreate(&t.a));
    CHK(hipEventCreate(&t.b));
    hipLaunchKernelGGL(k_philox, dim3(workgroups), dim3(kThreads), 0, nullptr, (uint32_t)n_draws, 7u, 0u, out,
                       clk);
    CHK(hipEventRecord(t.a, nullptr));
    hipLaunchKernelGGL(k_philox, dim3(workgroups), dim3(kThreads), 0, nullptr, (uint32_t)n_draws, 7u, 0u, out,
                       clk);
    CHK(hipEventRecord(t.b, nullptr));
    CHK(hipEventSynchronize(t.b));
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, t.a, t.b));
    *draws_per_s = (double)workgroups * kThreads * n_draws / (ms * 1e-3);
    unsigned long long* h = new unsigned long long[(size_t)workgroups * 2];
    const bool ok = hipMemcpy(h, clk, (size_t)workgroups * 16, hipMemcpyDeviceToHost) == hipSuccess;
    double cyc = 0.0, real = 0.0;
    for (int i = 0; ok && i < workgroups; ++i) {
        cyc += (double)h[2 * i];
        real += (double)h[2 * i + 1];
    }
    delete[] h;
    *clock_hz = real > 0 ? cyc / real * 1e8 : 0.0;  // s_memrealtime counts at 100 MHz
    CHK(hipFree(out));
    CHK(hipFree(clk));
    return ok ? 0 : -1;
}

// Microseconds per launch of an empty one-wave kernel: n back-to-back stream
// launches; the same n launches as hipGraph replays of a graph of
// `per_graph` kernels; and a launch the host waits for (hipStreamSynchronize
// after each, n_sync times).
int fcs_ceil_launch(int device, int n, int per_graph, int n_sync, double* us_plain, double* us_graph,
                    double* us_sync)
{
    if (n < 1 || per_graph < 1 || n % per_graph || n_sync < 1 || !us_plain || !us_graph || !us_sync) return -2;
    CHK(hipSetDevice(device));
    hipStream_t s = nullptr;
    CHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    Timer t;
    CHK(hipEventCreate(&t.a));
    CHK(hipEventCreate(&t.b));
    for (int i = 0; i < 100; ++i) hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s);
    CHK(hipStreamSynchronize(s));
    CHK(hipEventRecord(t.a, s));
    for (int i = 0; i < n; ++i) hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s);
    CHK(hipEventRecord(t.b, s));
    CHK(hipEventSynchronize(t.b));
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, t.a, t.b));
    *us_plain = ms * 1e3 / n;

    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    CHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < per_graph; ++i) hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s);
    CHK(hipStreamEndCapture(s, &g));
    CHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    CHK(hipGraphLaunch(ge, s));
    CHK(hipStreamSynchronize(s));
    CHK(hipEventRecord(t.a, s));
    for (int i = 0; i < n / per_graph; ++i) CHK(hipGraphLaunch(ge, s));
    CHK(hipEventRecord(t.b, s));
    CHK(hipEventSynchronize(t.b));
    CHK(hipEventElapsedTime(&ms, t.a, t.b));
    *us_graph = ms * 1e3 / n;
    (void)hipGraphExecDestroy(ge);
    (void)hipGraphDestroy(g);

    // host-visible round trips, timed on the host clock by the caller's
    // convention: events bracket the whole loop
    CHK(hipEventRecord(t.a, s));
    for (int i = 0; i < n_sync; ++i) {
        hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s);
        CHK(hipStreamSynchronize(s));
    }
    CHK(hipEventRecord(t.b, s));
    CHK(hipEventSynchronize(t.b));
    CHK(hipEventElapsedTime(&ms, t.a, t.b));
    *us_sync = ms * 1e3 / n_sync;
    CHK(hipStreamDestroy(s));
    return 0;
}

}  // extern "C"
