// Batched ensemble step: one persistent launch advances every grid of the
// batch by one time step.  The work of all grids is laid out as one sequence
// of (grid, strip, row) triples (grid-major), each strip weighted by its rows
// plus BATCH_FILL for the pipeline fill of a segment; block number L takes
// the L-th of gridDim.x equal contiguous pieces, so the load is balanced
// however uneven the grids are.  Blocks are numbered XCD by XCD (the
// hardware deals them out to the 8 XCDs in turn), so neighbouring pieces,
// which hold neighbouring strips, share an L2.  Each grid has its own constants (sizes,
// dt/tau, D + I, dx, dy, boundary conditions) in a device table; the
// velocity set, and so the inverse moment matrix, is shared.
#include <hip/hip_runtime.h>

#include <atomic>

#include "launch.hpp"
#include "step_wide.hpp"

namespace cdbm {

namespace {

template <typename S, bool VEC>
__global__ void __launch_bounds__(StripKernel<S>::NT) k_batch_step(const S* __restrict__ fin,
                                                         S* __restrict__ fout,
                                                         const KParams* __restrict__ Ks,
                                                         const int64_t* __restrict__ f_off,
                                                         const int64_t* __restrict__ work_start,
                                                         int ngrids) {
    using SK = StripKernel<S>;
    __shared__ __attribute__((aligned(16))) S F0[SK::F0_ELEMS];
    __shared__ __attribute__((aligned(16))) S F1[SK::F1_ELEMS];
    const int64_t total = work_start[ngrids];
    const int G = gridDim.x, b = blockIdx.x;   // block number L, XCD by XCD
    const int xq = G / 8, xr = G % 8, xcd = b % 8;
    const int L = xcd * xq + min(xcd, xr) + b / 8;
    const int64_t u1 = total * (L + 1) / G;
    int64_t u = total * L / G;
    int g = 0;
    while (u < u1) {
        while (work_start[g + 1] <= u) ++g;   // grids are visited in order
        const KParams& K = Ks[g];
        // strip s of grid g spans BATCH_FILL + ny positions: the pipeline fill
        // of a segment, then one position per row
        const int64_t len = (int64_t)K.ny + BATCH_FILL;
        const int64_t v = u - work_start[g];
        const int s = (int)(v / len);
        const int64_t p0 = (int64_t)s * len;
        const int64_t e = min(p0 + len, min(u1, work_start[g + 1]) - work_start[g]);
        const int ya = (int)max((int64_t)0, v - p0 - BATCH_FILL);
        const int yb = (int)max((int64_t)0, e - p0 - BATCH_FILL);
        if (ya < yb)
            SK::template run<VEC>(fin + f_off[g], fout + f_off[g], K, s * SK::TX, ya, yb, F0, F1);
        u = work_start[g] + e;
    }
}

}  // namespace

template <typename S>
int batch_blocks() {
    // resident blocks per compute unit (the same on every gfx950 device)
    static std::atomic<int> per_cu{0};
    int nb = per_cu.load(std::memory_order_relaxed);
    if (nb < 1) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_step<S, true>,
                                                         StripKernel<S>::NT, 0) != hipSuccess ||
            nb < 1)
            nb = 1;
        per_cu.store(nb, std::memory_order_relaxed);
    }
    return nb * device_cus();
}

template <typename S>
hipError_t launch_batch_step(const void* fin, void* fout, const KParams* Ks, const int64_t* f_off,
                             const int64_t* work_start, int ngrids, int nblocks, bool chunked,
                             hipStream_t st) {
    if (chunked && aligned16(fin, fout))
        hipLaunchKernelGGL((k_batch_step<S, true>), dim3(nblocks), dim3(StripKernel<S>::NT), 0, st,
                           (const S*)fin, (S*)fout, Ks, f_off, work_start, ngrids);
    else
        hipLaunchKernelGGL((k_batch_step<S, false>), dim3(nblocks), dim3(StripKernel<S>::NT), 0, st,
                           (const S*)fin, (S*)fout, Ks, f_off, work_start, ngrids);
    return hipGetLastError();
}

int strip_width(int precision) {
    return precision == CDBM_MIXED ? StripKernel<float>::TX : StripKernel<double>::TX;
}

template int batch_blocks<float>();
template int batch_blocks<double>();
template hipError_t launch_batch_step<float>(const void*, void*, const KParams*, const int64_t*,
                                             const int64_t*, int, int, bool, hipStream_t);
template hipError_t launch_batch_step<double>(const void*, void*, const KParams*, const int64_t*,
                                              const int64_t*, int, int, bool, hipStream_t);

}  // namespace cdbm
