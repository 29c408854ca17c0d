// Host memory for results and job copies: page-locked blocks, kept in a
// bounded cache when freed.  Device-to-host and host-to-device copies from
// page-locked memory go straight over the bus, and a reused block has no
// page faults, which on fresh memory cost more than the copy itself.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <map>
#include <mutex>
#include <unordered_map>

#include "hostmem.hpp"

namespace tp {
namespace {

constexpr size_t GRAIN = 2u << 20;          // block sizes are multiples of 2 MiB
constexpr size_t CACHE_LIMIT = 16ull << 30;  // bytes kept in freed blocks at most

struct Pool {
    std::mutex m;
    std::multimap<size_t, void *> free_blocks;  // size -> block
    std::unordered_map<void *, size_t> pinned;  // every live or cached pinned block
    size_t cached = 0;
};

Pool &pool() {
    static Pool *p = new Pool;  // never destroyed: blocks may be freed at exit
    return *p;
}

}  // namespace

void *host_alloc(size_t bytes) {
    if (bytes == 0)
        bytes = 1;
    const size_t size = (bytes + GRAIN - 1) / GRAIN * GRAIN;
    Pool &P = pool();
    {
        std::lock_guard<std::mutex> lk(P.m);
        // smallest cached block that fits, if not more than twice the need
        auto it = P.free_blocks.lower_bound(size);
        if (it != P.free_blocks.end() && it->first <= 2 * size) {
            void *b = it->second;
            P.cached -= it->first;
            P.free_blocks.erase(it);
            return b;
        }
    }
    void *b = nullptr;
    if (hipHostMalloc(&b, size, hipHostMallocDefault) == hipSuccess && b) {
        std::lock_guard<std::mutex> lk(P.m);
        P.pinned[b] = size;
        return b;
    }
    (void)hipGetLastError();  // not page-locked then: plain memory
    return std::malloc(bytes);
}

void host_free(void *b) {
    if (!b)
        return;
    Pool &P = pool();
    std::unique_lock<std::mutex> lk(P.m);
    auto it = P.pinned.find(b);
    if (it == P.pinned.end()) {
        lk.unlock();
        std::free(b);
        return;
    }
    const size_t size = it->second;
    if (P.cached + size <= CACHE_LIMIT) {
        P.free_blocks.emplace(size, b);
        P.cached += size;
        return;
    }
    P.pinned.erase(it);
    lk.unlock();
    (void)hipHostFree(b);
}

}  // namespace tp
