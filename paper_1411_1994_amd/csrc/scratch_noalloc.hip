// Static device scratch for the allocation-free shift-sum entry point (lsum_shift_sum_noalloc).
//
// Callers that cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc) still need the assembled 1D sums of Thm
// thm:sumCaseE (A).  That step needs device memory beyond its inputs and outputs: the job
// descriptor, the term list and up to two windowed strided sums of the reference rows.  Here
// they live in one file-scope device array of fixed size.  Its address is taken once per
// device with hipGetSymbolAddress (the array's name is only a host-side stand-in in host
// code) and kept per device; kernels receive that address.
//
// Every call on a device shares that device's array: calls that overlap on one device (on
// different streams or host threads) race.  Nothing in it needs clearing between calls: the
// descriptor and terms are copied in and the window tables are overwritten in full.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lsum_internal.h"

namespace lsum {

namespace {

__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

}  // namespace

int noalloc_scratch(int device, void** ptr) {
    if (device < 0 || device >= kMaxDevices) return fail(LSUM_E_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[device]) {
        // the caller has made `device` current: the address is that device's copy of the array
        void* p = nullptr;
        LSUM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LSUM_E_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        g_addr[device] = p;
    }
    *ptr = g_addr[device];
    return LSUM_OK;
}

}  // namespace lsum
