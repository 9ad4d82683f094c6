// Random-read probe: the rate at which the chip serves independent 16-byte
// reads at unrelated addresses of a buffer far larger than the caches.  The
// gather of the sector H.v issues one such read per off-diagonal term (the
// target's hash slot), so this rate, not the streaming bandwidth, is the
// ceiling that kernel is measured against.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ed_internal.hpp"

namespace ed {

// sink for the XOR of everything read: written only when it takes a value no
// read pattern produces in practice, so the loads cannot be removed and the
// probe writes nothing.  External linkage keeps the store (and with it the
// loads) from being discarded as unobservable.
__device__ unsigned long long g_probe_sink;

namespace {

// SplitMix64 finaliser (Steele, Lea and Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014): a counter-based 64-bit mixer.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// every lane reads iters slots of 16 B (W = 1) or 32 B (W = 2, two 16-byte
// loads of one 32-byte slot, as the complex H.v reads its slots) at
// pseudo-random slot-aligned offsets below (mask + 1) * 16 * W, two slots in
// flight
template <int W>
__global__ void __launch_bounds__(1024) k_probe_random_reads(const char *__restrict__ buf, uint64_t mask, int iters)
{
    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
    constexpr int kShift = W == 2 ? 5 : 4;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t h = splitmix64(tid * 0x100000001b3ull + 1u);
    uint64_t acc = 0;
    for (int it = 0; it < iters; it += 2) {
        const uint64_t a = splitmix64(h + (uint64_t)it) & mask;
        const uint64_t b = splitmix64(h + (uint64_t)it + 1u) & mask;
        const u64x2 va = *(const u64x2 *)(buf + (a << kShift));
        const u64x2 vb = *(const u64x2 *)(buf + (b << kShift));
        acc ^= va.x ^ va.y ^ vb.x ^ vb.y;
        if constexpr (W == 2) {
            const u64x2 wa = *(const u64x2 *)(buf + (a << kShift) + 16);
            const u64x2 wb = *(const u64x2 *)(buf + (b << kShift) + 16);
            acc ^= wa.x ^ wa.y ^ wb.x ^ wb.y;
        }
    }
    if (acc == 0x5bd1e9955bd1e995ull) g_probe_sink = acc;
}

}  // namespace

}  // namespace ed

extern "C" int ed_probe_random_reads(const void *buf_dev, int64_t bytes, int32_t slot_bytes, int32_t iters,
                                     int32_t reps, double *reads_per_s, void *stream)
{
    using namespace ed;
    if (!buf_dev || !reads_per_s) return set_error(ED_ERR_ARG, "null argument");
    if (slot_bytes != 16 && slot_bytes != 32) return set_error(ED_ERR_ARG, "slot_bytes = %d (16 or 32)", slot_bytes);
    if (bytes < (1 << 20) || (bytes & (bytes - 1))) return set_error(ED_ERR_ARG, "bytes = %lld (a power of two, >= 1 MiB)", (long long)bytes);
    if (iters < 2 || iters > 4096 || (iters & 1)) return set_error(ED_ERR_ARG, "iters = %d (even, 2..4096)", iters);
    if (reps < 1 || reps > 100) return set_error(ED_ERR_ARG, "reps = %d (1..100)", reps);
    hipStream_t st = (hipStream_t)stream;
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n_cu <= 0)
        return set_error(ED_ERR_HIP, "device query failed");
    const int threads = 1024, blocks = 2 * n_cu;   // two 1024-thread blocks per compute unit
    const uint64_t mask = (uint64_t)(bytes / slot_bytes) - 1u;
    auto kern = slot_bytes == 32 ? k_probe_random_reads<2> : k_probe_random_reads<1>;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return set_error(ED_ERR_HIP, "event creation failed");
    }
    int rc = ED_OK;
    // one untimed launch, then reps timed ones
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), 0, st, (const char *)buf_dev, mask, iters);
    if (hipEventRecord(e0, st) != hipSuccess) rc = set_error(ED_ERR_HIP, "event record failed");
    for (int r = 0; r < reps && rc == ED_OK; ++r)
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), 0, st, (const char *)buf_dev, mask, iters);
    if (rc == ED_OK && hipGetLastError() != hipSuccess) rc = set_error(ED_ERR_HIP, "probe launch failed");
    if (rc == ED_OK && hipEventRecord(e1, st) != hipSuccess) rc = set_error(ED_ERR_HIP, "event record failed");
    if (rc == ED_OK && hipEventSynchronize(e1) != hipSuccess)
        rc = set_error(ED_ERR_HIP, "probe failed: %s", hipGetErrorString(hipGetLastError()));
    float ms = 0.f;
    if (rc == ED_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = set_error(ED_ERR_HIP, "event timing failed");
    if (rc == ED_OK) *reads_per_s = (double)blocks * threads * iters * reps / (ms * 1e-3);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}
