// Batched ensemble step: one persistent launch advances every grid of the
// batch by one time step, in one of two work layouts.  Contiguous form: the
// work of all grids is laid out as one sequence of (grid, strip, row) triples
// (grid-major), each strip weighted by its rows plus `fill` positions for the
// pipeline fill of a segment; block number L takes
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
                                                         int ngrids, int fill) {
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
        // strip s of grid g spans fill + ny positions: the pipeline fill of a
        // segment, then one position per row
        const int64_t len = (int64_t)K.ny + fill;
        const int64_t v = u - work_start[g];
        const int s = (int)(v / len);
        const int64_t p0 = (int64_t)s * len;
        const int64_t e = min(p0 + len, min(u1, work_start[g + 1]) - work_start[g]);
        const int ya = (int)max((int64_t)0, v - p0 - fill);
        const int yb = (int)max((int64_t)0, e - p0 - fill);
        if (ya < yb)
            SK::template run<VEC>(fin + f_off[g], fout + f_off[g], K, s * SK::TX, ya, yb, F0, F1);
        u = work_start[g] + e;
    }
}

// Row-piece form.  The work is a table of units (grid, strip, first row,
// end row), built on the host: each grid cut into row pieces, numbered grid
// by grid, piece by piece, strip by strip, so that consecutive units are
// neighbouring strips of the same rows, and optionally each grid's last
// rows as smaller units after the pieces.  The table is cut into nq
// contiguous ranges of about equal weight (rows plus the pipeline fill),
// one per XCD; block b (on XCD b % 8) takes the units of range b % nq in
// order, one at a time, from that range's counter.  The blocks working at
// the same time on one XCD then hold neighbouring strips at the same rows
// (their row segments share DRAM pages, their halo lines that XCD's L2),
// and a block that finishes early takes the next unit.  Once its own range
// is used up a block takes units from the other ranges in turn, so that no
// XCD idles while another still has work; it leaves once every range is
// used up (each counter only grows, so one pass over the ranges suffices),
// and the last block to leave resets the counters for the next launch.
template <typename S, bool VEC>
__global__ void __launch_bounds__(StripKernel<S>::NT) k_batch_step_rows(
    const S* __restrict__ fin, S* __restrict__ fout, const KParams* __restrict__ Ks,
    const int64_t* __restrict__ f_off, const int4* __restrict__ units,
    const int64_t* __restrict__ range_start, int nq, int* __restrict__ counters) {
    using SK = StripKernel<S>;
    __shared__ __attribute__((aligned(16))) S F0[SK::F0_ELEMS];
    __shared__ __attribute__((aligned(16))) S F1[SK::F1_ELEMS];
    // the unit number is handed to the block through the first bytes of F0:
    // the rings are idle between units (a segment ends behind a barrier after
    // its last ring access and starts by writing F0 after the second barrier
    // below), and the two rings fill the whole 160 KiB of LDS
    volatile int64_t* s_u = reinterpret_cast<volatile int64_t*>(F0);
    const int q0 = blockIdx.x % nq;
    for (int k = 0; k < nq; ++k) {
        const int q = (q0 + k) % nq;
        const int64_t u_begin = range_start[q], u_end = range_start[q + 1];
        for (;;) {
            if (threadIdx.x == 0) *s_u = u_begin + atomicAdd(&counters[q], 1);
            __syncthreads();
            // the same value in every lane: make it scalar, so that everything
            // derived from it (grid, strip, rows) stays in scalar registers
            const int64_t ul = *s_u;
            const int64_t u = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(
                                             (int)(ul >> 32))
                                         << 32) |
                                        (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)ul));
            __syncthreads();   // every thread has read the unit before F0 is written again
            if (u >= u_end) break;
            const int4 t = units[u];
            const int g = __builtin_amdgcn_readfirstlane(t.x);
            const int x0 = __builtin_amdgcn_readfirstlane(t.y);
            const int ya = __builtin_amdgcn_readfirstlane(t.z);
            const int yb = __builtin_amdgcn_readfirstlane(t.w);
            SK::template run<VEC>(fin + f_off[g], fout + f_off[g], Ks[g], x0, ya, yb, F0, F1);
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&counters[nq], 1) == (int)gridDim.x - 1)
            for (int k = 0; k <= nq; ++k) atomicExch(&counters[k], 0);
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
                             const int64_t* work_start, int ngrids, int fill, int nblocks,
                             bool chunked, hipStream_t st) {
    if (chunked && aligned16(fin, fout))
        hipLaunchKernelGGL((k_batch_step<S, true>), dim3(nblocks), dim3(StripKernel<S>::NT), 0, st,
                           (const S*)fin, (S*)fout, Ks, f_off, work_start, ngrids, fill);
    else
        hipLaunchKernelGGL((k_batch_step<S, false>), dim3(nblocks), dim3(StripKernel<S>::NT), 0, st,
                           (const S*)fin, (S*)fout, Ks, f_off, work_start, ngrids, fill);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_batch_step_rows(const void* fin, void* fout, const KParams* Ks,
                                  const int64_t* f_off, const int* units,
                                  const int64_t* range_start, int nq, int* counters, int nblocks,
                                  bool chunked, hipStream_t st) {
    const int4* t = reinterpret_cast<const int4*>(units);
    if (chunked && aligned16(fin, fout))
        hipLaunchKernelGGL((k_batch_step_rows<S, true>), dim3(nblocks), dim3(StripKernel<S>::NT), 0,
                           st, (const S*)fin, (S*)fout, Ks, f_off, t, range_start, nq, counters);
    else
        hipLaunchKernelGGL((k_batch_step_rows<S, false>), dim3(nblocks), dim3(StripKernel<S>::NT),
                           0, st, (const S*)fin, (S*)fout, Ks, f_off, t, range_start, nq, counters);
    return hipGetLastError();
}

int strip_width(int precision) {
    return precision == CDBM_MIXED ? StripKernel<float>::TX : StripKernel<double>::TX;
}

template int batch_blocks<float>();
template int batch_blocks<double>();
template hipError_t launch_batch_step<float>(const void*, void*, const KParams*, const int64_t*,
                                             const int64_t*, int, int, int, bool, hipStream_t);
template hipError_t launch_batch_step<double>(const void*, void*, const KParams*, const int64_t*,
                                              const int64_t*, int, int, int, bool, hipStream_t);
template hipError_t launch_batch_step_rows<float>(const void*, void*, const KParams*,
                                                 const int64_t*, const int*, const int64_t*, int,
                                                 int*, int, bool, hipStream_t);
template hipError_t launch_batch_step_rows<double>(const void*, void*, const KParams*,
                                                  const int64_t*, const int*, const int64_t*, int,
                                                  int*, int, bool, hipStream_t);

}  // namespace cdbm
