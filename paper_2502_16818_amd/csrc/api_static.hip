// Entry point that allocates nothing: grid totals with the block partial
// sums in a statically allocated device array instead of a handle's buffer.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/cdbm.h"
#include "api_internal.hpp"
#include "launch.hpp"
#include "model.hpp"

namespace cdbm {

// Partial sums of the totals reduction: 4 doubles for each of its
// REDUCE_BLOCKS blocks (32 KiB).  One copy per GPU, held until the process
// ends; every call on a GPU shares it.
constexpr int STATIC_PARTIALS = 4 * REDUCE_BLOCKS;
static __device__ __align__(256) double scratch[STATIC_PARTIALS];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mutex;
double* g_scratch[MAX_DEVICES] = {};   // device address of `scratch` on each GPU

// Address of this GPU's `scratch` (the host-side name is not a device
// address), looked up once per device with that device current.
int scratch_address(int dev, double** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return fail(CDBM_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress of the static scratch");
        g_scratch[dev] = (double*)p;
    }
    *out = g_scratch[dev];
    return CDBM_OK;
}

}  // namespace
}  // namespace cdbm

using namespace cdbm;

extern "C" int cdbm_conserved_totals_static(const cdbm_params* p, const void* f, double* out4,
                                            void* stream) {
    if (!p || !f || !out4) return fail(CDBM_EINVAL, "null argument");
    KParams K;
    std::string err;
    int rc = build_params(*p, K, err);
    if (rc != CDBM_OK) return fail(rc, err);
    static_assert(STATIC_PARTIALS >= 4 * REDUCE_BLOCKS, "the static scratch holds every partial");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    double* part = nullptr;
    rc = scratch_address(dev, &part);
    if (rc != CDBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    e = p->precision == CDBM_MIXED_COMP ? launch_totals_comp(f, part, REDUCE_BLOCKS, out4, K, st)
        : p->precision == CDBM_MIXED    ? launch_totals<float>(f, part, REDUCE_BLOCKS, out4, K, st)
                                        : launch_totals<double>(f, part, REDUCE_BLOCKS, out4, K, st);
    return e == hipSuccess ? CDBM_OK : hip_fail(e, "totals launch");
}
