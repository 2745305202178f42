// Fused CDBM time step on one grid: a persistent launch whose blocks each
// take an equal, contiguous share of the grid's (strip, row) sequence, so
// that every block streams down as few strips as possible and the work is
// balanced to within a few rows.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "step_fused.hpp"

namespace cdbm {

namespace {

template <typename S, bool VEC>
__global__ void __launch_bounds__(FusedGeom<S>::NT) k_step_fused(const S* __restrict__ fin,
                                                                 S* __restrict__ fout,
                                                                 const KParams* __restrict__ Kd) {
    __shared__ __attribute__((aligned(16))) S F0[FusedGeom<S>::F0_ELEMS];
    __shared__ __attribute__((aligned(16))) S F1[FusedGeom<S>::F1_ELEMS];
    const KParams& K = *Kd;
    const int nstrips = (K.nx + FUSED_TX - 1) / FUSED_TX;
    // Block b takes the b-th of gridDim.x equal, contiguous pieces of the
    // strip-major sequence of (strip, row) pairs.
    const int64_t work = (int64_t)nstrips * K.ny;
    const int64_t u1 = work * (blockIdx.x + 1) / gridDim.x;
    int64_t u = work * blockIdx.x / gridDim.x;
    while (u < u1) {
        const int s = (int)(u / K.ny);
        const int ya = (int)(u - (int64_t)s * K.ny);
        const int yb = (int)min((int64_t)K.ny, (int64_t)ya + (u1 - u));
        fused_strip<S, VEC>(fin, fout, K, s * FUSED_TX, ya, yb, F0, F1);
        u += yb - ya;
    }
}

template <typename S>
int fused_grid_blocks(const KParams& K) {
    static int per_cu = -1, cus = -1;
    if (per_cu < 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 256;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
        cus = prop.multiProcessorCount;
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_fused<S, true>, FusedGeom<S>::NT, 0) !=
                hipSuccess ||
            nb < 1)
            nb = 1;
        per_cu = nb;
    }
    const int nstrips = (K.nx + FUSED_TX - 1) / FUSED_TX;
    const int64_t work = (int64_t)nstrips * K.ny;
    int64_t g = (int64_t)per_cu * cus;
    // each block should stream at least ~32 rows so the pipeline warm-up stays small
    const int64_t cap = (work + 31) / 32;
    if (g > cap) g = cap;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

template <typename S>
hipError_t launch_step_fused(const void* fin, void* fout, const KParams& K, const KParams* Kd,
                             hipStream_t st) {
    const int g = fused_grid_blocks<S>(K);
    if (fused_chunked<S>(K.nx, fin, fout))
        hipLaunchKernelGGL((k_step_fused<S, true>), dim3(g), dim3(FusedGeom<S>::NT), 0, st,
                           (const S*)fin, (S*)fout, Kd);
    else
        hipLaunchKernelGGL((k_step_fused<S, false>), dim3(g), dim3(FusedGeom<S>::NT), 0, st,
                           (const S*)fin, (S*)fout, Kd);
    return hipGetLastError();
}

template hipError_t launch_step_fused<float>(const void*, void*, const KParams&, const KParams*,
                                             hipStream_t);
template hipError_t launch_step_fused<double>(const void*, void*, const KParams&, const KParams*,
                                              hipStream_t);

}  // namespace cdbm
