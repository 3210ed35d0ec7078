// Replay of captured launch sequences from HIP graphs.
//
// A launch sequence (kernels only: no memsets, copies or host synchronisation)
// is recorded on a private capture stream of the current device, turned into
// a graph and launched on the caller's stream.  Instantiated graphs are kept
// per thread (a few per thread, most recent first); a new capture with the
// same shape (same kernels in the same order) only refreshes the kernel
// arguments of a kept one through hipGraphExecUpdate, so a sequence that is
// re-captured with new pointers or scalars costs no new instantiation; a
// sequence whose caller-supplied key (all its arguments, as bytes) equals a
// kept graph's is replayed without capturing at all.
#include <mutex>
#include <string>
#include <vector>

#include "ndq_solver.h"

namespace ndq {
namespace {

constexpr size_t kKeep = 4;
constexpr int kMaxDevices = 64;

struct Kept {
    int device;
    hipGraphExec_t exec;
    std::string key;
};

thread_local std::vector<Kept> t_kept;

std::mutex g_mu;
hipStream_t g_capture[kMaxDevices] = {};

int capture_stream(int dev, hipStream_t* out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(NDQ_EINVAL, "graph: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_capture[dev]) NDQ_HIP(hipStreamCreateWithFlags(&g_capture[dev], hipStreamNonBlocking));
    *out = g_capture[dev];
    return NDQ_OK;
}

}  // namespace

int launch_captured(const std::function<int(hipStream_t)>& body, hipStream_t st, const std::string& key) {
    int dev = 0;
    NDQ_HIP(hipGetDevice(&dev));
    if (!key.empty()) {
        // the same launch sequence with the same arguments: replay as it is
        for (size_t k = 0; k < t_kept.size(); ++k) {
            if (t_kept[k].device == dev && t_kept[k].key == key) {
                const Kept hit = t_kept[k];
                t_kept.erase(t_kept.begin() + (long)k);
                t_kept.insert(t_kept.begin(), hit);
                NDQ_HIP(hipGraphLaunch(hit.exec, st));
                return NDQ_OK;
            }
        }
    }
    hipStream_t cs = nullptr;
    int rc = capture_stream(dev, &cs);
    if (rc) return rc;
    NDQ_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    rc = body(cs);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (rc || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc ? rc : fail(NDQ_EHIP, "graph: capture failed: %s", hipGetErrorString(ec));
    }
    hipGraphExec_t exec = nullptr;
    for (size_t k = 0; k < t_kept.size(); ++k) {
        if (t_kept[k].device != dev) continue;
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        const hipError_t eu = hipGraphExecUpdate(t_kept[k].exec, graph, &err_node, &res);
        if (eu == hipSuccess && res == hipGraphExecUpdateSuccess) {
            exec = t_kept[k].exec;
            t_kept[k].key = key;
            const Kept hit = t_kept[k];
            t_kept.erase(t_kept.begin() + (long)k);
            t_kept.insert(t_kept.begin(), hit);
            break;
        }
        (void)hipGetLastError();   // a shape mismatch is not an error here
    }
    if (!exec) {
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(NDQ_EHIP, "graph: instantiate failed: %s", hipGetErrorString(ei));
        }
        t_kept.insert(t_kept.begin(), Kept{dev, exec, key});
        if (t_kept.size() > kKeep) {
            // the evicted graph may still run on some stream of this device
            NDQ_HIP(hipDeviceSynchronize());
            (void)hipGraphExecDestroy(t_kept.back().exec);
            t_kept.pop_back();
        }
    }
    (void)hipGraphDestroy(graph);
    NDQ_HIP(hipGraphLaunch(exec, st));
    return NDQ_OK;
}

}  // namespace ndq
