// opf_eval_set_noalloc: the callback set of opf_eval_set for callers that
// cannot allocate device memory (code under HIP graph capture, serving
// loops, harnesses that forbid hipMalloc).  Its kernels are opf_eval_set's;
// only their scratch (objective partials, the one-launch arrival ticket and
// the half-edge records) moves from the model's own arena into one
// file-scope device array of fixed size, shared by every call on a device.
#include <mutex>

#include "internal.h"

namespace {

// The shared scratch.  In host code `scratch` names a host-side stand-in,
// not device memory: the device address comes from hipGetSymbolAddress,
// once per device, and only that address is ever handed to a kernel.
constexpr size_t kNoAllocScratch = size_t(OPF_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) char scratch[kNoAllocScratch];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device `dev`.
int scratch_ptr(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return opf_internal::set_err(OPF_E_ARG, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) return opf_internal::hip_err(e, "hipGetSymbolAddress(scratch)");
        g_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_ptr[dev];
    return OPF_OK;
}

// Zeroes the arrival ticket: a fill kernel rather than hipMemsetAsync, so
// that the call can be captured into a graph and replayed.
__global__ void clear_ticket(int32_t* ticket) { *ticket = 0; }

}  // namespace

extern "C" int opf_eval_set_noalloc(opf_model m, const double* x, const double* y, double obj_weight, double* f,
                                    double* g, double* c, double* jvals, double* hvals, void* stream) {
    using namespace opf_internal;
    if (!valid_model(m)) return set_err(OPF_E_STATE, "invalid or destroyed model handle");
    if (!x) return set_err(OPF_E_ARG, "x must be non-NULL");
    if (hvals && !y) return set_err(OPF_E_ARG, "y must be non-NULL when hvals is requested");
    const size_t need = opf::scratch_bytes(m->dm);
    if (need > kNoAllocScratch)
        return set_err(OPF_E_ARG, "model needs %zu bytes of scratch; opf_eval_set_noalloc has %zu", need,
                       kNoAllocScratch);
    DeviceGuard dg(m->device);
    if (dg.err != hipSuccess) return hip_err(dg.err, "hipSetDevice");
    char* base = nullptr;
    if (int rc = scratch_ptr(m->device, &base)) return rc;
    opf::DevModel d = m->dm;
    attach_scratch(d, base);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (d.single && f) hipLaunchKernelGGL(clear_ticket, dim3(1), dim3(1), 0, s, d.obj_ticket);
    opf::EvalOut o{};
    o.x = x;
    o.y = y;
    o.sigma = obj_weight;
    o.f = f;
    o.g = g;
    o.c = c;
    o.J = jvals;
    o.H = hvals;
    hipError_t e = opf::launch_eval_set(d, o, s);
    if (e != hipSuccess) return hip_err(e, "callback kernel launch");
    return OPF_OK;
}
