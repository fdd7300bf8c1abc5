// noalloc.hip -- lbm_adjoint_noalloc: the discrete adjoint with its scratch
// in a device array of the library instead of a caller workspace.
//
// For callers that cannot allocate device memory at the point of the call
// (code under stream capture, tight training or serving loops, harnesses
// that forbid allocation).  The scratch is a file-scope __device__ array of
// LBM_NOALLOC_SCRATCH_BYTES; every GPU the library is loaded on holds its
// own copy until the process ends.  Its device address is looked up once per
// device (hipGetSymbolAddress, with that device current) on the first call
// made there and kept in a host table; host code only ever passes that
// address on, never the array's name, which in host code is a stand-in and
// not a device address.
//
// All calls on one GPU share that GPU's array.  Calls ordered on one stream
// are fine; calls that overlap in time on one GPU (other streams, other
// threads) race on it.
#include <mutex>

#include "lbm_host.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[LBM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

// Device address of `scratch` on device dev; looked up on the first call
// for that device with dev current (the caller's current device is kept).
int scratch_on(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices)
        return lbm::fail(LBM_EDEVICE, "device ordinal out of the supported range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        int cur = -1;
        LBM_HIP(hipGetDevice(&cur));
        if (cur != dev) LBM_HIP(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) LBM_HIP(hipSetDevice(cur));
        if (e != hipSuccess || !p)
            return lbm::fail(LBM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                              hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return LBM_OK;
}

}  // namespace

extern "C" int lbm_adjoint_noalloc(lbm_ctx* c, int32_t seed_kind, const void* seed_dev,
                                   int64_t T, int64_t K, const void* ckpt_dev,
                                   void* grad_phi_dev, void* grad_drho_dev, void* lam0_dev) {
    if (!c) return lbm::fail(LBM_EINVAL, "NULL argument");
    // the context's device is the device of its stream
    int dev = -1;
    LBM_HIP(hipStreamGetDevice(c->stream, &dev));
    const size_t need = lbm_adjoint_workspace_bytes(c, K);
    if (need == 0)
        return lbm::fail(LBM_EINVAL, "the adjoint is implemented for single D2Q9 lattices (K >= 1)");
    if (need > (size_t)LBM_NOALLOC_SCRATCH_BYTES)
        return lbm::fail(LBM_ENOMEM,
                         "lbm_adjoint_noalloc: this lattice and K need " + std::to_string(need) +
                             " bytes of scratch, above the static " +
                             std::to_string((size_t)LBM_NOALLOC_SCRATCH_BYTES) +
                             " (use a smaller K or lbm_adjoint with a workspace)");
    void* work = nullptr;
    const int rc = scratch_on(dev, &work);
    if (rc != LBM_OK) return rc;
    return lbm::adjoint_entry(c, seed_kind, seed_dev, T, K, ckpt_dev, work,
                              (size_t)LBM_NOALLOC_SCRATCH_BYTES, grad_phi_dev, grad_drho_dev,
                              lam0_dev);
}
