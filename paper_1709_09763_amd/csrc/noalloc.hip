// Entry points that allocate nothing, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  Their
// scratch is a file-scope device array of fixed size; every GPU the library
// runs on holds one copy of it until the process ends.
#include <mutex>

#include "common.h"

namespace mls {

// prefix sums of the quantised weights of multinomial resampling (Sec. 2.4):
// one uint64 per particle
constexpr int64_t kNoAllocMaxN = int64_t(1) << 20;
static __device__ __align__(256) uint64_t scratch[kNoAllocMaxN];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint64_t* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device.  In host code the array's name is only a stand-in for the symbol:
// kernels must be given this address.
static int scratch_address(uint64_t** out)
{
    int dev = -1;
    MLS_CHECK_HIP(hipGetDevice(&dev));
    MLS_REQUIRE(dev >= 0 && dev < kMaxDevices, "noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        MLS_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        MLS_REQUIRE(p != nullptr, "noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = static_cast<uint64_t*>(p);
    }
    *out = g_scratch_ptr[dev];
    return MLS2MC_OK;
}

}  // namespace mls

using namespace mls;

extern "C" int mls2mc_resample_noalloc(int64_t N, const double* w, const double* u, int32_t* anc_out,
                                       void* stream)
{
    MLS_REQUIRE(N >= 1 && N <= kNoAllocMaxN,
                "resample_noalloc: need 1 <= N <= 2^20 (the size of the library's static scratch)");
    MLS_REQUIRE(w && u && anc_out, "resample_noalloc: null pointer");
    uint64_t* C = nullptr;
    MLS_TRY(scratch_address(&C));
    return launch_resample_into(N, w, u, C, anc_out, (hipStream_t)stream);
}
