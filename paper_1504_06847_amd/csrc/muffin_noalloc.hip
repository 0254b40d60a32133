// muffin_grad_noalloc: the reverse sweep of muffin_grad with its scratch in
// a file-scope device array instead of a workspace the caller attaches, for
// callers that cannot allocate device memory.  Every GPU the library runs on
// holds its own copy of the array (kNoAllocScratchBytes) until the process
// ends; calls on one GPU share it, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "muffin.h"
#include "muffin_ctx.hpp"

namespace {

constexpr size_t kNoAllocScratchBytes = size_t(MUFFIN_NOALLOC_SCRATCH_MIB) << 20;

}  // namespace

// Device scratch of muffin_grad_noalloc.  In host code this name is a host-side
// stand-in, not a device address: host code uses the per-device address that
// hipGetSymbolAddress returns (scratch_on) and never the name itself.
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_scratch[kMaxDevices];

// The address of `scratch` on device `dev`, looked up once per device with
// that device current (the previous current device is restored).
int scratch_on(int dev, char** out) {
    std::lock_guard<std::mutex> guard(g_lock);
    if (dev < 0 || dev >= kMaxDevices) {
        muffin::set_error("muffin_grad_noalloc: device %d outside the %d the library tracks", dev, kMaxDevices);
        return MUFFIN_EDEVICE;
    }
    if (!g_scratch[dev]) {
        int cur = 0;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) HIP_TRY(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) HIP_TRY(hipSetDevice(cur));
        if (e != hipSuccess || !p) {
            muffin::set_error("muffin_grad_noalloc: hipGetSymbolAddress of the static scratch failed: %s",
                              hipGetErrorString(e));
            return MUFFIN_EDEVICE;
        }
        g_scratch[dev] = p;
    }
    *out = (char*)g_scratch[dev];
    return MUFFIN_OK;
}

}  // namespace

extern "C" int muffin_grad_noalloc(muffin_ctx* c, int K, int ckpt_every, const void* sky_or_gx, int mode,
                                   double* loss, double grad[3]) {
    using namespace muffin;
    if (int rc = grad_args(c, K, ckpt_every, sky_or_gx, mode, grad, "muffin_grad_noalloc")) return rc;
    const size_t need = grad_scratch_bytes(c, K, ckpt_every, false);
    if (need > kNoAllocScratchBytes) {
        set_error("muffin_grad_noalloc: the reverse sweep of %d passes with checkpoints every %d needs %zu "
                  "bytes of scratch; the static scratch holds %zu (MUFFIN_NOALLOC_SCRATCH_MIB MiB): use a "
                  "smaller spacing or muffin_grad with a workspace",
                  K, ckpt_every, need, kNoAllocScratchBytes);
        return MUFFIN_EWORKSPACE;
    }
    // the device the context's arrays live on
    hipPointerAttribute_t attr;
    HIP_TRY(hipPointerGetAttributes(&attr, c->ws));
    char* g = nullptr;
    if (int rc = scratch_on(attr.device, &g)) return rc;
    // passes launched one by one: recording a graph (muffin_set_graph) could
    // allocate; the launched form gives the same results bit for bit
    const int graph = c->use_graph;
    c->use_graph = 0;
    double full[7];
    const int rc = grad_sweep(c, K, ckpt_every, sky_or_gx, mode, loss, full, nullptr, g, kNoAllocScratchBytes);
    c->use_graph = graph;
    if (rc) return rc;
    grad[0] = full[1];
    grad[1] = full[2];
    grad[2] = full[3] + full[4] + full[5] + full[6];
    return MUFFIN_OK;
}
