// Allocation-free measurement of the exact height moments (W^2, Sec. 2.1,
// Eq. `eq:Wdef`) of a packed lattice in caller-owned device memory, for
// callers that cannot allocate device memory: code under stream capture,
// tight serving loops, harnesses that forbid allocation.
//
// The three measurement kernels of okpz_measure (column anchors, per-band
// integer moments, exact 128-bit totals) run unchanged; their intermediate
// buffers (the L column-0 anchors and the per-band partial sums) live in one
// file-scope device array, `scratch`, sized for the largest lattice the
// library takes (L = 2^17: 512 KiB of anchors and 1.5 MiB of partials).  Each
// device holds its own copy of the array for the life of the process.  Host
// code never uses the array's name as an address: the device address of
// each device's copy is looked up once, with that device current, by
// hipGetSymbolAddress, and passed to the kernels.
//
// Every call on a device shares that device's array, so calls that overlap
// on one device (two streams, or two host threads) race and give undefined
// results; calls on one stream are ordered.  Every word of scratch a call
// reads is written earlier in the same call, so nothing needs clearing.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

using namespace okpz;
using namespace okpz_host;

namespace {

constexpr uint32_t kNoAllocMaxL = 1u << 17;
constexpr size_t kAnchorBytes = (size_t)kNoAllocMaxL * sizeof(int32_t);
constexpr size_t kPartialBytes = (size_t)(kNoAllocMaxL / 4) * kMomentFields * sizeof(int64_t);
constexpr size_t kScratchBytes = kAnchorBytes + kPartialBytes;  // 2 MiB

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];  // device address of each device's copy of scratch

// The current device's copy of scratch (looked up on the first call there).
int scratch_address(void **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail_with(OKPZ_EINVAL, "okpz_measure_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail_with(OKPZ_EHIP, "okpz_measure_noalloc: no device address for the scratch array");
        g_scratch_addr[dev] = ptr;
    }
    *out = g_scratch_addr[dev];
    return OKPZ_OK;
}

}  // namespace

extern "C" int okpz_measure_noalloc(const void *dev_words, uint32_t L, void *hip_stream, int64_t *dev_totals,
                                    okpz_moments *out)
{
    if (!dev_words || !dev_totals || ((uintptr_t)dev_totals & 7u))
        return fail_with(OKPZ_EINVAL, "okpz_measure_noalloc: null or misaligned buffer");
    if (!is_pow2(L) || L < 64 || L > kNoAllocMaxL)
        return fail_with(OKPZ_EINVAL, "okpz_measure_noalloc: L must be a power of two in [64, 2^17]");
    void *base = nullptr;
    const int rc = scratch_address(&base);
    if (rc != OKPZ_OK) return rc;
    int32_t *h0 = static_cast<int32_t *>(base);
    int64_t *partial = reinterpret_cast<int64_t *>(static_cast<unsigned char *>(base) + kAnchorBytes);
    const hipStream_t st = (hipStream_t)hip_stream;
    const uint32_t *words = static_cast<const uint32_t *>(dev_words);
    const uint32_t nbx_log2 = ilog2(L / 32);
    const uint32_t rows_per_block = kMeasureThreads / 64;
    const uint32_t blocks = (L / 4 + rows_per_block - 1) / rows_per_block;
    // the partials region first holds the column-0 bytes (one per band)
    uint8_t *col0 = reinterpret_cast<uint8_t *>(partial);
    hipLaunchKernelGGL(col0_kernel, dim3((L / 4 + 255) / 256), dim3(256), 0, st, words, L, nbx_log2, col0);
    hipLaunchKernelGGL(anchors_kernel, dim3(1), dim3(1024), 0, st, col0, L, h0);
    hipLaunchKernelGGL((rows_kernel<false>), dim3(blocks), dim3(kMeasureThreads), 0, st, words, h0, nullptr,
                       nullptr, L, nbx_log2, partial);
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kReduceThreads), 0, st, partial, L / 4, dev_totals);
    HIP_TRY(hipGetLastError());
    if (out) {
        int64_t totals[2 * kMomentFields];
        HIP_TRY(hipMemcpyAsync(totals, dev_totals, sizeof(totals), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        moments_from_totals(L, 0, totals, out);
    }
    return OKPZ_OK;
}
