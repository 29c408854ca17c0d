// tp_run_noalloc: the caller-memory run (tp_run_ws) with the library's own
// fixed workspace, for callers that cannot allocate device memory.
//
// The workspace is a file-scope device array of TP_NOALLOC_WORKSPACE_MAX
// bytes.  Each GPU the library runs on holds its own copy at its own address
// from module load until the process ends.  In host code the array's name
// is only a stand-in for that address, so the address is looked up once per
// device (hipGetSymbolAddress, with that device current) and only that
// pointer is ever handed to kernels or copies.  Every call on a GPU shares
// the array: a call rewrites the layout tables and clears every counter,
// filter and table it uses, so the previous call's contents never matter,
// but calls that overlap on one GPU race on it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "runtime.hpp"

using namespace tp;

static_assert(TP_NOALLOC_WORKSPACE_MAX % 256 == 0, "whole 256-byte rows");

static __device__ __align__(256) uint8_t scratch[TP_NOALLOC_WORKSPACE_MAX];

namespace {

std::mutex g_scratch_mu;
std::vector<uint8_t *> g_scratch_ptr;  // per device: the array's device address

// The address of this device's scratch array (looked up on first use).
int scratch_of(int dev, uint8_t **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((size_t)dev >= g_scratch_ptr.size())
        g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                        hipGetErrorString(e));
        g_scratch_ptr[dev] = (uint8_t *)p;
    }
    *out = g_scratch_ptr[dev];
    return TP_OK;
}

}  // namespace

extern "C" int tp_run_noalloc(tp_plan *p, const uint8_t *d_input, void *d_outputs, void *stream) {
    if (!p)
        return fail(TP_EINVAL, "plan is NULL");
    if (!p->ws.valid || p->ws.gen != p->layout_gen)
        return fail(TP_ESTATE, "the plan has no current workspace layout "
                               "(tp_plan_workspace_layout)");
    if (p->ws.pub.workspace_bytes > TP_NOALLOC_WORKSPACE_MAX)
        return fail(TP_EINVAL, "the plan's workspace needs " +
                                   std::to_string(p->ws.pub.workspace_bytes) +
                                   " bytes; the fixed workspace holds " +
                                   std::to_string((uint64_t)TP_NOALLOC_WORKSPACE_MAX));
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    uint8_t *base = nullptr;
    int rc = scratch_of(dev, &base);
    if (rc)
        return rc;
    const hipStream_t s = (hipStream_t)stream;
    rc = ws_prepare(p, base, s);
    if (rc)
        return rc;
    return ws_run(p, d_input, base, (uint8_t *)d_outputs, s);
}
