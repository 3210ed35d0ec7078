// D_N^m applied with the library's own device scratch instead of a caller
// workspace, for callers that cannot allocate device memory.
//
// The scratch is one file-scope device array per GPU, of a fixed size, that
// lives until the process ends.  Host code never uses the array's name as an
// address: on the first call on each device (with that device current) its
// device address is looked up once with hipGetSymbolAddress and kept per
// device; every later call hands that address to the same arena the
// workspace-taking entry point uses, so the kernels and their arguments are
// the same as there.  Nothing in the workspace has to start at zero: every
// partial sum, device scalar and vector is written before it is read.
#include <hip/hip_runtime.h>
#include <string.h>

#include <chrono>
#include <mutex>

#include "ndq_solver.h"

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;   // 32 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device).
int scratch_ptr(void** out) {
    int dev = 0;
    NDQ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return ndq::fail(NDQ_EINVAL, "ndq_apply_DN_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        NDQ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return ndq::fail(NDQ_EHIP, "ndq_apply_DN_noalloc: no address for the scratch array");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return NDQ_OK;
}

}  // namespace

extern "C" {

size_t ndq_noalloc_scratch_bytes(void) { return kScratchBytes; }

int ndq_apply_DN_noalloc(const ndq_geom* g, const ndq_gauge* U, const ndq_overlap_params* p, const ndq_spinor* in,
                         const ndq_spinor* out, ndq_stats* stats, void* stream) {
    if (!g || !p || !p->approx || !in) return ndq::fail(NDQ_EINVAL, "ndq_apply_DN_noalloc: NULL argument");
    if (p->graph) return ndq::fail(NDQ_EINVAL, "ndq_apply_DN_noalloc: graph replay builds graph objects; set graph = 0");
    const size_t need = ndq_workspace_bytes(g, p, in->prec, NDQ_OP_DN);
    if (need == 0) return ndq::fail(NDQ_EINVAL, "ndq_apply_DN_noalloc: invalid parameters");
    if (need > kScratchBytes)
        return ndq::fail(NDQ_ENOMEM, "ndq_apply_DN_noalloc: needs %zu bytes of scratch, the static scratch holds %zu",
                         need, kScratchBytes);
    void* ws = nullptr;
    const int rc = scratch_ptr(&ws);
    if (rc) return rc;
    return ndq_apply_DN(g, U, p, in, out, ws, kScratchBytes, stats, stream);
}

}  // extern "C"
