// Fused CDBM time step on one grid: one launch per step, each block
// streaming down strips of the grid (step_fused.hpp, step_wide.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "launch.hpp"
#include "step_two.hpp"
#include "step_wide.hpp"

namespace cdbm {

namespace {

// pieces > 0: block number L < nstrips * pieces takes strip L % nstrips and
// the (L / nstrips)-th row piece of `len` rows (len = main_len, or ny /
// pieces rounded up when main_len is 0), so that blocks on neighbouring
// strips stream the same rows at the same time (their row segments share
// DRAM pages).  With main_len > 0 the pieces end at row pieces * main_len
// and the remaining rows of every strip (its tail) go to the blocks past
// nstrips * pieces: tail block j takes the tails of strips j, j + ntail,
// j + 2 ntail, ... in turn, so the tail blocks also work on neighbouring
// strips at the same time.
// Blocks are numbered XCD by XCD (the hardware deals them out to the 8 XCDs
// in turn), so the blocks of one XCD hold consecutive strips and read the
// halo columns they share through that XCD's L2 once.
// pieces == 0: block b takes the b-th of gridDim.x equal, contiguous pieces of
// the strip-major sequence of (strip, row) pairs.
template <typename S, bool VEC>
__global__ void __launch_bounds__(StripKernel<S>::NT) k_step_fused(const S* __restrict__ fin,
                                                                   S* __restrict__ fout,
                                                                   const KParams* __restrict__ Kd,
                                                                   int pieces, int main_len) {
    using SK = StripKernel<S>;
    __shared__ __attribute__((aligned(16))) S F0[SK::F0_ELEMS];
    __shared__ __attribute__((aligned(16))) S F1[SK::F1_ELEMS];
    const KParams& K = *Kd;
    const int nstrips = (K.nx + SK::TX - 1) / SK::TX;
    if (pieces > 0) {
        // blocks go to the 8 XCDs round-robin; number them XCD by XCD so that
        // the blocks of one XCD take consecutive strips of the same rows and
        // share the halo columns in that XCD's L2
        const int G = gridDim.x, b = blockIdx.x;
        const int xq = G / 8, xr = G % 8, xcd = b % 8;
        const int L = xcd * xq + min(xcd, xr) + b / 8;
        const int main_blocks = nstrips * pieces;
        const int len = main_len > 0 ? main_len : (K.ny + pieces - 1) / pieces;
        if (L < main_blocks) {
            const int s = L % nstrips, p = L / nstrips;
            const int ya = min(K.ny, p * len), yb = min(K.ny, (p + 1) * len);
            if (ya < yb) SK::template run<VEC>(fin, fout, K, s * SK::TX, ya, yb, F0, F1);
        } else {
            const int ntail = G - main_blocks, y0 = pieces * len;
            for (int s = L - main_blocks; s < nstrips && y0 < K.ny; s += ntail)
                SK::template run<VEC>(fin, fout, K, s * SK::TX, y0, K.ny, F0, F1);
        }
        return;
    }
    // this block's range [u, u1) of the strip-major sequence of (strip, row)
    const int64_t work = (int64_t)nstrips * K.ny;
    int64_t u = work * blockIdx.x / gridDim.x;
    const int64_t u1 = work * (blockIdx.x + 1) / gridDim.x;
    while (u < u1) {
        const int s = (int)(u / K.ny);
        const int ya = (int)(u - (int64_t)s * K.ny);
        const int yb = (int)min((int64_t)K.ny, (int64_t)ya + (u1 - u));
        SK::template run<VEC>(fin, fout, K, s * SK::TX, ya, yb, F0, F1);
        u += yb - ya;
    }
}

// Two steps per launch (step_two.hpp): the same block -> (strip, rows)
// mapping as k_step_fused, on strips of TwoStepGeom::TX columns.
template <bool VEC>
__global__ void __launch_bounds__(TwoStepGeom::NT) k_step2_fused(const float* __restrict__ fin,
                                                                float* __restrict__ fout,
                                                                const KParams* __restrict__ Kd,
                                                                int pieces, int main_len) {
    using G = TwoStepGeom;
    __shared__ __attribute__((aligned(16))) float F0[G::RING_ELEMS];
    __shared__ __attribute__((aligned(16))) float F1[G::RING_ELEMS];
    __shared__ __attribute__((aligned(16))) float F2[G::RING_ELEMS];
    __shared__ __attribute__((aligned(16))) float F3[G::RING_ELEMS];
    const KParams& K = *Kd;
    const int nstrips = (K.nx + G::TX - 1) / G::TX;
    if (pieces > 0) {
        const int Gn = gridDim.x, b = blockIdx.x;
        const int xq = Gn / 8, xr = Gn % 8, xcd = b % 8;
        const int L = xcd * xq + min(xcd, xr) + b / 8;
        const int main_blocks = nstrips * pieces;
        const int len = main_len > 0 ? main_len : (K.ny + pieces - 1) / pieces;
        if (L < main_blocks) {
            const int s = L % nstrips, p = L / nstrips;
            const int ya = min(K.ny, p * len), yb = min(K.ny, (p + 1) * len);
            if (ya < yb) fused_strip_2<VEC>(fin, fout, K, s * G::TX, ya, yb, F0, F1, F2, F3);
        } else {
            const int ntail = Gn - main_blocks, y0 = pieces * len;
            for (int s = L - main_blocks; s < nstrips && y0 < K.ny; s += ntail)
                fused_strip_2<VEC>(fin, fout, K, s * G::TX, y0, K.ny, F0, F1, F2, F3);
        }
        return;
    }
    const int64_t work = (int64_t)nstrips * K.ny;
    int64_t u = work * blockIdx.x / gridDim.x;
    const int64_t u1 = work * (blockIdx.x + 1) / gridDim.x;
    while (u < u1) {
        const int s = (int)(u / K.ny);
        const int ya = (int)(u - (int64_t)s * K.ny);
        const int yb = (int)min((int64_t)K.ny, (int64_t)ya + (u1 - u));
        fused_strip_2<VEC>(fin, fout, K, s * G::TX, ya, yb, F0, F1, F2, F3);
        u += yb - ya;
    }
}

struct Launch {
    int blocks, pieces, main_len;
};

// Grid of the step: row-aligned pieces.  Plain form: P equal row
// pieces per strip, one block per (strip, piece), in as many rounds of one
// block per compute unit as nstrips * P needs; P minimises rounds * (rows
// per piece + fill), the time of the busiest compute unit with the pipeline
// fill of every piece counted as `fill` rows (FILL_ROWS for the one-step
// strips, FILL_ROWS_TWO for the two-step strip; at 8192 x 8192:
// 11 pieces in three rounds, 15 % faster than one round).  Tail form, for
// one round with compute units to spare (nstrips * P < CUs): P pieces of L
// rows per strip and the remaining T = ny - P L rows of each strip on the
// spare units, k = ceil(nstrips / spare) tails on the busiest one; L
// minimises max(L + fill, k (T + fill)) (4096 x 4096 in FP32: 35
// strips of 120 columns, 7 pieces of 567 rows and 11 units taking 3 or 4 tails of 127 rows, against
// 7 pieces of 586 rows and 11 idle units; FP64, 74 strips of 56 columns:
// 3 pieces of 1232 rows and 34 units taking 2 or 3 tails of 400 rows).  The
// launch takes the cheaper form.  A persistent grid that splits the
// strip-major sequence of (strip, row) evenly over the compute units
// balances the rows exactly but loses the row alignment of neighbouring
// strips and their shared halo lines in L2 (18 % slower at 4096 x 4096 in
// FP32, 1 % in FP64, whose step is bound more by latency: one wave per row,
// 6 waves per compute unit); it serves grids too short for pieces of 32
// rows.
constexpr int FILL_ROWS = 12;
// The two-step strip fills a pipeline four stages deep: 16 halo rows.
constexpr int FILL_ROWS_TWO = 24;

Launch strip_launch(const KParams& K, int TX, int fill) {
    const int cus = device_cus();   // one block per compute unit (LDS-bound)
    const int nstrips = (K.nx + TX - 1) / TX;
    const int pmax = K.ny / 32;   // rows per piece stay >= 32
    if (pmax >= 1) {
        // the search runs on every launch of a handle: remember the last grid
        thread_local int last_nx = -1, last_ny = -1, last_cus = -1, last_tx = -1;
        thread_local Launch last{1, 1, 0};
        if (K.nx == last_nx && K.ny == last_ny && cus == last_cus && TX == last_tx) return last;
        Launch best{nstrips, 1, 0};
        int64_t best_cost = -1;
        for (int p = 1; p <= pmax; ++p) {
            const int64_t blocks = (int64_t)nstrips * p;
            if (blocks > (int64_t)1 << 30) break;
            const int64_t rounds = (blocks + cus - 1) / cus;
            const int64_t cost = rounds * ((K.ny + p - 1) / p + fill);
            if (best_cost < 0 || cost < best_cost) {
                best_cost = cost;
                best = Launch{(int)blocks, p, 0};
            }
            const int64_t spare = cus - blocks;
            if (spare <= 0) continue;
            // tail form: the crossing of L + F and k (ny - p L + F), rounded
            // both ways
            const int64_t k = (nstrips + spare - 1) / spare;
            const int64_t l0 = (k * (K.ny + fill) - fill) / (1 + k * p);
            for (int64_t l = l0; l <= l0 + 1; ++l) {
                const int64_t t = K.ny - p * l;
                if (l < 32 || t < 1) continue;
                const int64_t c = std::max(l + fill, k * (t + fill));
                if (c < best_cost) {
                    best_cost = c;
                    best = Launch{(int)(blocks + std::min<int64_t>(spare, nstrips)), p, (int)l};
                }
            }
        }
        last_nx = K.nx;
        last_ny = K.ny;
        last_cus = cus;
        last_tx = TX;
        last = best;
        return best;
    }
    const int64_t work = (int64_t)nstrips * K.ny;
    int64_t g = std::min<int64_t>(cus, (work + 31) / 32);
    return Launch{(int)(g < 1 ? 1 : g), 0, 0};
}

template <typename S>
Launch fused_launch(const KParams& K) {
    return strip_launch(K, StripKernel<S>::TX, FILL_ROWS);
}

}  // namespace

int device_cus() {
    constexpr int MAX_DEVICES = 64;
    static std::atomic<int> cache[MAX_DEVICES] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return 256;
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n > 0) return n;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess || prop.multiProcessorCount < 1)
        return 256;
    n = prop.multiProcessorCount;
    cache[dev].store(n, std::memory_order_relaxed);
    return n;
}

template <typename S>
hipError_t launch_step_fused(const void* fin, void* fout, const KParams& K, const KParams* Kd,
                             hipStream_t st) {
    const Launch l = fused_launch<S>(K);
    if (fused_chunked<S>(K.nx, K.ny, fin, fout))
        hipLaunchKernelGGL((k_step_fused<S, true>), dim3(l.blocks), dim3(StripKernel<S>::NT), 0, st,
                           (const S*)fin, (S*)fout, Kd, l.pieces, l.main_len);
    else
        hipLaunchKernelGGL((k_step_fused<S, false>), dim3(l.blocks), dim3(StripKernel<S>::NT), 0,
                           st, (const S*)fin, (S*)fout, Kd, l.pieces, l.main_len);
    return hipGetLastError();
}

hipError_t launch_step2_fused(const void* fin, void* fout, const KParams& K, const KParams* Kd,
                              hipStream_t st) {
    const Launch l = strip_launch(K, TwoStepGeom::TX, FILL_ROWS_TWO);
    if (fused_chunked<float>(K.nx, K.ny, fin, fout))
        hipLaunchKernelGGL((k_step2_fused<true>), dim3(l.blocks), dim3(TwoStepGeom::NT), 0, st,
                           (const float*)fin, (float*)fout, Kd, l.pieces, l.main_len);
    else
        hipLaunchKernelGGL((k_step2_fused<false>), dim3(l.blocks), dim3(TwoStepGeom::NT), 0, st,
                           (const float*)fin, (float*)fout, Kd, l.pieces, l.main_len);
    return hipGetLastError();
}

template hipError_t launch_step_fused<float>(const void*, void*, const KParams&, const KParams*,
                                             hipStream_t);
template hipError_t launch_step_fused<double>(const void*, void*, const KParams&, const KParams*,
                                              hipStream_t);

}  // namespace cdbm
