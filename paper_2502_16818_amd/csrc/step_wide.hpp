// Fused two-stage Runge-Kutta step with FP32 storage on wide strips.
//
// Same pipeline as fused_strip (step_fused.hpp), with a strip of TX = 120
// output columns handled by two waves per row (64 columns each) and R = 6
// rows per iteration, so that a block still has 12 waves:
//   F0: f^n rows, TX + 8 = 128 columns;  F1: f^(1) rows, TX + 4 = 124 columns
//   stored at a stride of 128;  ring depth R + 4 = 10 rows each (160 KB of
//   LDS, all of it).  With both strides at 512 bytes the rows of successive
//   velocities are two 256-byte steps apart, so every LDS read of a cell's
//   16 velocities (and every store of its f^(1)) uses one base address and
//   paired reads with immediate offsets; the 124-float stride needed an
//   address computation every other velocity.
// A row of f^n is fetched from HBM as 16 contiguous 512-byte segments (one
// per velocity), and stage 1 is recomputed on 4 halo columns for 120 outputs.
// Wave (r, h) of a row r computes columns [62h - 1, 62h + 63) of the
// strip's stage-1 and stage-2 windows and keeps its lanes 1 .. 62: the
// x-direction NND takes the neighbouring cells' minmod terms from the
// neighbouring lanes (stage_cell_k with XLANE).  The global loads of the next rows are issued
// in two halves, before stage 1 and before stage 2, and each lane stores its
// own stage-2 cell: spreading the memory instructions over the iteration
// keeps waves from stalling on a full memory queue.
#pragma once

#include "step_fused.hpp"

namespace cdbm {

struct WideGeom {
    static constexpr int TX = 120;           // output columns per strip
    static constexpr int WPR = 2;            // waves per row
    static constexpr int R = 6;              // rows per iteration
    static constexpr int W0 = TX + 8;        // F0 row width
    static constexpr int W1 = TX + 8;        // F1 row stride (TX + 4 columns used)
    static constexpr int SLOTS = R + 4;
    static constexpr int NT = R * WPR * 64;
    static constexpr int F0_ELEMS = SLOTS * NV * W0;
    static constexpr int F1_ELEMS = SLOTS * NV * W1;
    static_assert(W0 == 64 * WPR && W1 <= 64 * WPR, "one column per lane");
};

// Advance rows [ya, yb) of the strip starting at column x0.  All threads of
// the block call this together.  VEC selects the 16-byte-chunk form (see
// fused_strip); fused_chunked<float> must hold for it.
template <bool VEC>
__device__ __forceinline__ void fused_strip_w(const float* __restrict__ fin,
                                              float* __restrict__ fout, const KParams& K, int x0,
                                              int ya, int yb, float* F0, float* F1) {
    using S = float;
    using V = Chunk<float>::type;
    using G = WideGeom;
    constexpr int R = G::R, SLOTS = G::SLOTS, W0 = G::W0, W1 = G::W1, TX = G::TX;
    constexpr int CW = 4;
    constexpr int LCH = W0 / CW;                  // 32 chunks per loaded velocity row
    constexpr int NLD = NV * LCH / (64 * G::WPR); // 4 chunk loads per lane and row
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rw = wave >> 1;                     // row of the iteration, uniform
    const int h = wave & 1;                       // half of the row, uniform
    const int col = 64 * h + lane;                // column of this lane in the F0 row (loads)
    // Column of this lane in the stage windows.  The x-direction NND shares
    // minmod terms between neighbouring lanes, so the first and last lane of
    // each wave only serve their neighbours: wave h computes columns
    // 62h - 1 .. 62h + 62 and keeps lanes 1 .. 62.
    const int ccol = 62 * h - 1 + lane;
    const bool keep = lane >= 1 && lane <= 62;
    const int nx = K.nx, ny = K.ny, bcx = K.bcx, bcy = K.bcy;
    const int64_t cells = (int64_t)nx * ny;
    const int nrows = yb - ya;

    auto slot = [&](int q) { return (q + 4 * SLOTS) % SLOTS; };

    // Chunked form.  A row has NV * 32 loaded chunks (velocity c / 32,
    // columns x0 - 4 + 4 (c % 32) ..); wave half h moves chunks
    // c = 256h + 64k + lane, k < NLD, which land at element 4c of the row's F0
    // slot.  Their velocity is 8h + 2k + (lane >> 5) and their column does not
    // depend on k, so one per-lane byte offset ld_lane serves all of them.
    const uint32_t plane = (uint32_t)(cells * (int64_t)sizeof(S));   // bytes per velocity plane
    uint32_t ld_lane = 0;
    if constexpr (VEC) {
        int cs = x0 - 4 + 4 * (lane & 31);
        if (cs < 0 || cs >= nx) {   // periodic image (zero-gradient ghosts are never read)
            cs %= nx;
            if (cs < 0) cs += nx;
        }
        ld_lane = (uint32_t)(lane >> 5) * plane + (uint32_t)cs * (uint32_t)sizeof(S);
    }
    // per-column form: global column this lane loads
    const int gc = VEC ? 0 : map_index(x0 - 4 + col, nx, bcx);

    // the two waves of row rw load row 4 + (t-2)R + rw at iteration t
    constexpr int NPRE = VEC ? NLD : NV;
    using P = typename std::conditional<VEC, V, S>::type;
    P pre[NPRE];
    auto load_row = [&](int t) { return 4 + (t - 2) * R + rw; };
    auto wanted = [&](int q) { return q >= -4 && q < nrows + 4; };
    // loads of part `half` (0 or 1) of the row of iteration t
    auto issue_loads = [&](int t, int half) {
        const int q = load_row(t);
        if (!wanted(q)) return;
        const S* src = fin + (int64_t)source_row(ya + q, ny, bcy) * nx;
        if constexpr (VEC) {
            const char* base = (const char*)src;
#pragma unroll
            for (int k = 0; k < NLD; ++k)
                if (k / (NLD / 2) == half)
                    pre[k] = *(const V*)(base + (uint32_t)(8 * h + 2 * k) * plane + ld_lane);
        } else {
#pragma unroll
            for (int i = 0; i < NV; ++i)
                if (i / (NV / 2) == half) pre[i] = src[(int64_t)i * cells + gc];
        }
    };
    // called at iteration t, for the rows of that iteration
    auto store_loads = [&](int t) {
        const int q = load_row(t);
        if (!wanted(q)) return;
        S* dst = F0 + slot(q) * NV * W0;
        if constexpr (VEC) {
#pragma unroll
            for (int k = 0; k < NLD; ++k) *(V*)(dst + 4 * (256 * h + 64 * k + lane)) = pre[k];
        } else {
#pragma unroll
            for (int i = 0; i < NV; ++i) dst[i * W0 + col] = pre[i];
        }
    };

    const int t0 = 2 - (8 + R - 1) / R;          // first iteration whose loads reach row -4
    const int t_end = (nrows + R - 1) / R + 1;   // last iteration with a stage-2 row
    // Iteration t runs stage 1 (phase A), then stores the f^n rows that
    // stage 1 of t + 1 needs and runs stage 2 (phase B): two barriers per
    // iteration.  The F0 slots that phase B refills held the rows of this
    // iteration's stage-2 cells, so stage 1 reads those cells' f^n (the Heun
    // term) into registers first.
    issue_loads(t0, 0);
    issue_loads(t0, 1);
    store_loads(t0);
    issue_loads(t0 + 1, 0);
    lds_barrier();   // the previous segment of this block is done with the rings
    S fn2[NV];       // f^n of this lane's stage-2 cell
    for (int t = t0; t <= t_end; ++t) {
        if (t < t_end) issue_loads(t + 1, 1);
        // phase A, stage 1: f^(1) at row q1, column x0 - 2 + ccol
        const int q1 = 2 + (t - 2) * R + rw;
        const int q2 = q1 - 2;   // stage-2 row of this iteration
        if (q1 >= -2 && q1 < nrows + 2) {
            RingLd<S, W0> ld;
            ld.ring = F0;
            const int x1 = x0 - 2 + ccol;
#pragma unroll
            for (int o = -2; o <= 2; ++o) {
                ld.slot[o + 2] = slot(q1 + o);
                const int c = (bcx == CDBM_ZERO_GRADIENT) ? min(max(x1 + o, 0), nx - 1) - (x0 - 4)
                                                          : ccol + 2 + o;
                ld.col[o + 2] = min(max(c, 0), W0 - 1);   // discarded lanes read in bounds
            }
            S out[NV];
            stage_cell_k<S, false, RingLd<S, W0>, true>(ld, K, out);
#pragma unroll
            for (int i = 0; i < NV; ++i) materialize(out[i]);
            if (keep && ccol < TX + 4) {
                S* dst = F1 + slot(q1) * NV * W1 + ccol;
#pragma unroll
                for (int i = 0; i < NV; ++i) dst[i * W1] = out[i];
            }
            if (q2 >= 0 && q2 < nrows) {
                const S* fn = F0 + slot(q2) * NV * W0 + min(4 + ccol, W0 - 1);
#pragma unroll
                for (int i = 0; i < NV; ++i) fn2[i] = fn[i * W0];
            }
        }
        lds_barrier();

        // phase B: f^n rows for stage 1 of t + 1, then stage 2
        if (t < t_end) {
            store_loads(t + 1);
            if (t + 1 < t_end) issue_loads(t + 2, 0);
        }
        // stage 2: f^{n+1} at row q2, column x0 + ccol
        if (q2 >= 0 && q2 < nrows) {
            const int r2 = ya + q2;
            const int x = x0 + ccol;
            RingLd<S, W1> ld;
            ld.ring = F1;
#pragma unroll
            for (int o = -2; o <= 2; ++o) {
                const int rr = (bcy == CDBM_ZERO_GRADIENT) ? min(max(r2 + o, 0), ny - 1) : r2 + o;
                const int cc = (bcx == CDBM_ZERO_GRADIENT) ? min(max(x + o, 0), nx - 1) : x + o;
                ld.slot[o + 2] = slot(rr - ya);
                ld.col[o + 2] = min(max(cc - (x0 - 2), 0), W1 - 1);
            }
            S out[NV];
            stage_cell_k<S, true, RingLd<S, W1>, true>(ld, K, out);
#pragma unroll
            for (int i = 0; i < NV; ++i) materialize(out[i]);
            if (keep && ccol < TX && x < nx) {
                S* dst = fout + (int64_t)r2 * nx + x;
#pragma unroll
                for (int i = 0; i < NV; ++i) dst[(int64_t)i * cells] = fma(S(0.5), fn2[i], out[i]);
            }
        }
        lds_barrier();   // stage 1 of t + 1 overwrites F1 slots read above
    }
}

}  // namespace cdbm

namespace cdbm {

// The strip kernel of each storage type: FP32 uses the wide strip, FP64
// (twice the LDS per row) the 56-column strip of fused_strip.
template <typename S>
struct StripKernel;
template <>
struct StripKernel<float> {
    static constexpr int TX = WideGeom::TX, NT = WideGeom::NT;
    static constexpr int F0_ELEMS = WideGeom::F0_ELEMS, F1_ELEMS = WideGeom::F1_ELEMS;
    template <bool VEC>
    static __device__ __forceinline__ void run(const float* fin, float* fout, const KParams& K,
                                               int x0, int ya, int yb, float* F0, float* F1) {
        fused_strip_w<VEC>(fin, fout, K, x0, ya, yb, F0, F1);
    }
};
template <>
struct StripKernel<double> {
    using G = FusedGeom<double>;
    static constexpr int TX = G::TX, NT = G::NT;
    static constexpr int F0_ELEMS = G::F0_ELEMS, F1_ELEMS = G::F1_ELEMS;
    template <bool VEC>
    static __device__ __forceinline__ void run(const double* fin, double* fout, const KParams& K,
                                               int x0, int ya, int yb, double* F0, double* F1) {
        fused_strip<double, VEC>(fin, fout, K, x0, ya, yb, F0, F1);
    }
};

}  // namespace cdbm
