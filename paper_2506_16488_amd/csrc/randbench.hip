// Random-access reference rates of the device, for the benchmark's second
// roofline: the round kernel is bound by scattered 8-16 byte accesses to
// the search state, whose achievable rate is far below streaming bandwidth.
//
// This is a measurement probe built into its own library (libppsp_probe.so),
// outside the search library and its C interface. probe_randbench(device,
// words, accesses, kind, ms) times one kernel that performs `accesses`
// operations at
// pseudo-random 16-byte-aligned positions of a table of `words` 64-bit words
// (positions from a counter hash, so every run is the same):
//   kind 0: 16-byte loads (the state pair of a vertex), summed per thread
//   kind 1: 64-bit atomicMin at device scope (the WriteMin of a relaxation)
// and returns the kernel time (HIP events) of the second of two runs in *ms.
// Returns 0, or -1 for bad arguments (null ms, words < 2 or > 2^40,
// accesses == 0, kind not 0/1), -3 when the table cannot be allocated, -7 on
// a HIP error.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppsp_randbench_kernels {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_rand_load(const ulonglong2 *t, uint64_t pairs, uint64_t per, uint64_t *sink) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t acc = 0;
    for (uint64_t k = 0; k < per; k++) {
        const ulonglong2 v = t[mix64(tid * per + k + 0x9E3779B97F4A7C15ull) % pairs];
        acc += v.x ^ v.y;
    }
    if (acc == 0x5A5A5A5A5A5A5A5Aull) sink[0] = acc;   // keeps the loads; practically never stores
}

__global__ __launch_bounds__(256) void k_rand_atomic(unsigned long long *t, uint64_t words, uint64_t per) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t k = 0; k < per; k++) {
        const uint64_t h = mix64(tid * per + k + 0x632BE59BD9B4E019ull);
        atomicMin(t + (h % words), h >> 1);
    }
}

}  // namespace ppsp_randbench_kernels

using namespace ppsp_randbench_kernels;

extern "C" int probe_randbench(int device, uint64_t words, uint64_t accesses, int kind, double *ms) {
    enum { E_INVALID = -1, E_OOM = -3, E_DEVICE = -7 };
    if (!ms || words < 2 || accesses == 0 || kind < 0 || kind > 1 || words > (1ull << 40)) return E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return E_DEVICE;
    words &= ~1ull;
    void *t = nullptr, *sink = nullptr;
    if (hipMalloc(&t, words * 8) != hipSuccess) return E_OOM;
    if (hipMalloc(&sink, 8) != hipSuccess) { (void)hipFree(t); return E_OOM; }
    int rc = 0;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    (void)hipMemset(t, 0x7F, words * 8);
    const uint32_t threads = 256, blocks = 8192;
    const uint64_t per = (accesses + (uint64_t)threads * blocks - 1) / ((uint64_t)threads * blocks);
    for (int rep = 0; rep < 2 && rc == 0; rep++) {   // the first run warms up
        (void)hipEventRecord(a, nullptr);
        if (kind == 0)
            k_rand_load<<<blocks, threads>>>((const ulonglong2 *)t, words / 2, per, (uint64_t *)sink);
        else
            k_rand_atomic<<<blocks, threads>>>((unsigned long long *)t, words, per);
        if (hipGetLastError() != hipSuccess) { rc = E_DEVICE; break; }
        (void)hipEventRecord(b, nullptr);
        if (hipEventSynchronize(b) != hipSuccess) rc = E_DEVICE;
        float f = 0;
        (void)hipEventElapsedTime(&f, a, b);
        *ms = f;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(t);
    (void)hipFree(sink);
    return rc;
}
