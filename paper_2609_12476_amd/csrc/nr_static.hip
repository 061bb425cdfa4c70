// The segment sum without device allocation: every buffer of the plan is
// carved from one static scratch array per GPU (see
// nufft_resample_semicoherent_sum_static in include/nufft_resample.h).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/nufft_resample.h"
#include "nr_internal.hpp"

namespace {

constexpr int kMaxDevices = 64;

// The scratch array.  In host code its name is only a host-side stand-in:
// its device address on each GPU comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address is used.
static __device__ __align__(256) unsigned char scratch[NR_STATIC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch (NULL with *err set on failure).
void* scratch_of_current_device(hipError_t* err, int* device)
{
    *err = hipGetDevice(device);
    if (*err != hipSuccess) return nullptr;
    if (*device < 0 || *device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[*device]) {
        void* ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*err != hipSuccess || !ptr) {
            if (*err == hipSuccess) *err = hipErrorInvalidSymbol;
            return nullptr;
        }
        g_scratch_ptr[*device] = ptr;
    }
    return g_scratch_ptr[*device];
}

}  // namespace

extern "C" {

nr_status nufft_resample_semicoherent_sum_static(const nr_segment* segs, int32_t n_segs,
                                                 const nr_template* tmpls, int32_t n_tmpls,
                                                 const nr_instance* inst, int64_t n_inst, double tol,
                                                 const nr_options* opt, const void* strain,
                                                 const double* seg_weight, void* stat, int32_t* n_used)
{
    hipError_t e = hipSuccess;
    int device = -1;
    void* base = scratch_of_current_device(&e, &device);
    if (!base) {
        // the message goes where nufft_resample_last_error(NULL) reads it
        return nr::report_create_error(NR_ERR_DEVICE, std::string("static scratch of device ") +
                                                          std::to_string(device) + ": " + hipGetErrorString(e));
    }
    return nr::semicoherent_sum_in_arena(base, NR_STATIC_SCRATCH_BYTES, segs, n_segs, tmpls, n_tmpls, inst, n_inst,
                                         tol, opt, strain, seg_weight, stat, n_used);
}

}  // extern "C"
