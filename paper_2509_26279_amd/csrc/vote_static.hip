// sas_vote_static: sas_vote for callers that cannot allocate device memory.
//
// sas_vote keeps its scratch (the window index of the catalog, the per-
// detection cell ids and ranks, the staged positions, the refinement list)
// in a caller workspace.  This variant keeps it in `scratch`, one file-scope
// device array of kStaticScratchBytes per GPU, instead.  Host code never
// passes the array's name to a kernel (on the host it names a stand-in, not
// device memory): the first call on each device looks up the array's
// device address with hipGetSymbolAddress, with that device current, and
// every launch takes that address.  The array lives until the process ends.
//
// Every call on one GPU shares its array, and the vote clears what must
// start at zero itself (the preparation's counters, the refinement
// counter), so a call needs nothing from the one before.  Calls that overlap
// on one GPU (two streams, or two threads) race on the array.
#include <mutex>
#include <string>

#include "internal.h"

namespace sas {
void set_error(const std::string &msg);
}

namespace {

sas_status sfail(sas_status s, const std::string &m) {
    sas::set_error(m);
    return s;
}

sas_status shipfail(hipError_t e, const char *what) {
    return sfail(SAS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr size_t kStaticScratchBytes = (size_t)SAS_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// Device address of this device's scratch array (looked up once per device,
// with the device current); null with the error in *err on failure.
void *scratch_of_device(int dev, hipError_t *err) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    *err = hipSuccess;
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" sas_status sas_vote_static(const sas_plan *p, const int32_t *x_q8,
                                      const int32_t *y_q8, const uint8_t *epoch, int64_t n,
                                      sas_candidate *cand_dev, int64_t cand_cap,
                                      sas_vote_result *res_dev, void *stream) {
    if (!p) return sfail(SAS_E_INVALID, "sas_vote_static: null plan");
    if (n < 0) return sfail(SAS_E_INVALID, "sas_vote_static: n must be >= 0");
    size_t need = 0;
    sas_status st = sas_vote_workspace_size(p, n, &need);
    if (st != SAS_OK) return st;
    if (need > kStaticScratchBytes)
        return sfail(SAS_E_WORKSPACE,
                         "sas_vote_static: this plan and catalog need " + std::to_string(need) +
                             " bytes of scratch, more than the static maximum of " +
                             std::to_string(kStaticScratchBytes) +
                             "; use sas_vote with a workspace (or a smaller tuning.refine_cap)");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return shipfail(e, "sas_vote_static: no device");
    if (dev < 0 || dev >= kMaxDevices)
        return sfail(SAS_E_UNSUPPORTED, "sas_vote_static: device ordinal above 63");
    void *ws = scratch_of_device(dev, &e);
    if (!ws) return shipfail(e, "sas_vote_static: looking up the scratch array");
    return sas_vote(p, x_q8, y_q8, epoch, n, cand_dev, cand_cap, res_dev, ws,
                    kStaticScratchBytes, stream);
}
