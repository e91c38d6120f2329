// The step entry point that allocates nothing (slw_step_noalloc): its
// statistics counters and the workspace that permutes v_in into the
// internal order live in one static device array of this file instead of
// the context's counters and its grow-on-demand workspace.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "slw_internal.h"

namespace {

// [0, 256): the counters (DevStats); [256, kScratchBytes): the workspace
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr size_t kCountersBytes = 256;
static_assert(sizeof(slw::DevStats) <= kCountersBytes, "counters fit their slot");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device (each GPU holds its own copy
// of the array at its own address).  The array's name in host code is a
// host-side stand-in, never a device address: kernels and copies get the
// resolved address only.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

}  // namespace

namespace slw {

slw_status noalloc_init(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return set_error(SLW_E_UNSUPPORTED, "device index beyond the no-allocation scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_addr[device])
        return SLW_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return set_error(SLW_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_addr[device] = p;
    return SLW_OK;
}

}  // namespace slw

extern "C" slw_status slw_step_noalloc(slw_mesh *mesh, const slw_field *field, double t_n, double dt, int scheme,
                                       int order, int start_mode, const int32_t *start, const void *v_in, int vdtype,
                                       int k, void *v_out, double outside_value, int32_t *elem, slw_stats *stats_h)
{
    if (!mesh)
        return slw::set_error(SLW_E_ARG, "slw_step_noalloc: mesh is NULL");
    const int dev = mesh->ctx->device;
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        base = (dev >= 0 && dev < kMaxDevices) ? g_addr[dev] : nullptr;
    }
    if (!base)  // resolved by slw_ctx_create for the context's device
        return slw::set_error(SLW_E_HIP, "slw_step_noalloc: scratch address of the device not resolved");
    slw::StepScratch sc;
    sc.stats = (slw::DevStats *)base;
    sc.work = (unsigned char *)base + kCountersBytes;
    sc.work_bytes = kScratchBytes - kCountersBytes;
    return slw::step_impl(mesh, field, t_n, dt, scheme, order, start_mode, start, v_in, vdtype, k, v_out,
                          outside_value, elem, stats_h, sc, "slw_step_noalloc");
}
