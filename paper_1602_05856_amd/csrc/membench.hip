// Random-access rate of the memory system, for the roofline of the
// junction-finding kernels (a measurement aid, not part of the method).
//
// The fill, the query, the record and the decision each make one random
// access per position into a filter or a table; their ceiling is the rate
// at which the chip serves random 8-byte accesses into a structure of a
// given size -- from the L2 and the 256 MB last-level cache when it fits
// there, from HBM (through the address translation) when it does not.  This
// kernel makes the same kind of accesses with nothing else to do: every
// thread draws its addresses from a counter-based hash (no index stream
// from memory), keeps several loads in flight, and folds every loaded word
// into a checksum that it writes out, so no load can be dropped.
#include <algorithm>

#include "device.hpp"
#include "runtime.hpp"

namespace tp {

constexpr uint32_t MB_INFLIGHT = 8;  // independent accesses per thread per step

template <int MODE>
__global__ __launch_bounds__(BLOCK) void k_random_access(uint64_t *buf, uint64_t words,
                                                         uint64_t per_thread, uint64_t seed,
                                                         unsigned long long *checksum) {
    const uint64_t tid = blockIdx.x * (uint64_t)BLOCK + threadIdx.x;
    uint64_t acc = 0;
    for (uint64_t i = 0; i < per_thread; i += MB_INFLIGHT) {
        uint64_t idx[MB_INFLIGHT], v[MB_INFLIGHT];
#pragma unroll
        for (uint32_t j = 0; j < MB_INFLIGHT; ++j) {
            const uint64_t h = mix64(seed ^ (tid * 0x9E3779B97F4A7C15ull + i + j));
            idx[j] = __umul64hi(h, words);  // uniform in [0, words)
        }
#pragma unroll
        for (uint32_t j = 0; j < MB_INFLIGHT; ++j) {
            if (MODE == 0) {
                v[j] = __hip_atomic_load((unsigned long long *)&buf[idx[j]], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
            } else {
                // the fill's read-modify-write: an atomic OR of one bit
                v[j] = __hip_atomic_fetch_or((unsigned long long *)&buf[idx[j]],
                                             1ull << (idx[j] & 63), __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < MB_INFLIGHT; ++j)
            acc ^= v[j] + idx[j];
    }
    if (acc)
        atomicXor(checksum, (unsigned long long)acc);
}

}  // namespace tp

using namespace tp;

extern "C" int tp_bench_random_access(void *d_buf, uint64_t bytes, uint64_t accesses,
                                      uint32_t mode, uint64_t seed, uint64_t *d_checksum,
                                      void *stream, uint64_t *accesses_done) {
    if (!d_buf || !d_checksum || !accesses_done || bytes < 8 || mode > 1)
        return fail(TP_EINVAL, "random access bench: bad arguments");
    if ((uintptr_t)d_buf % 8 || (uintptr_t)d_checksum % 8)
        return fail(TP_EINVAL, "random access bench: buffers must be 8-byte aligned");
    int dev = 0, ncu = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const uint64_t grid = (uint64_t)std::max(1, ncu) * 8;
    const uint64_t threads = grid * BLOCK;
    const uint64_t per_thread =
        std::max<uint64_t>(MB_INFLIGHT, (accesses + threads - 1) / threads / MB_INFLIGHT *
                                            MB_INFLIGHT);
    const hipStream_t s = (hipStream_t)stream;
    if (mode == 0)
        hipLaunchKernelGGL(k_random_access<0>, dim3((uint32_t)grid), dim3(BLOCK), 0, s,
                           (uint64_t *)d_buf, bytes / 8, per_thread, seed,
                           (unsigned long long *)d_checksum);
    else
        hipLaunchKernelGGL(k_random_access<1>, dim3((uint32_t)grid), dim3(BLOCK), 0, s,
                           (uint64_t *)d_buf, bytes / 8, per_thread, seed,
                           (unsigned long long *)d_checksum);
    HIPCHK(hipGetLastError());
    *accesses_done = threads * per_thread;
    return TP_OK;
}
