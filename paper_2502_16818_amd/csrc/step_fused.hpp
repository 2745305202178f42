// Fused two-stage Runge-Kutta step of the CDBM (both stages in one pass
// over HBM).
//
// A block owns a strip of TX = 60 output columns and streams down the grid
// in y, R = 4 rows per iteration, keeping two ring buffers in LDS:
//   F0: f^n rows, 2R slots of TX + 8 columns (x halo of 4 each side);
//   F1: f^(1) = f^n + dt L(f^n) rows, 2R slots of TX + 4 columns.
// Iteration t (rows relative to the strip start y0):
//   load  f^n  rows [y0 - 4 + tR,   y0 - 4 + (t+1)R)   (global -> registers -> F0)
//   stage 1    rows [y0 - 2 + (t-1)R, y0 - 2 + tR)      (F0 -> F1; one cell per thread)
//   stage 2    rows [y0 + (t-2)R,   y0 + (t-1)R)        (F1, F0 -> f^{n+1} in HBM)
// so each f value crosses HBM once in and once out per step; stage 1 is
// recomputed only on the 2-column x halo (64 columns for 60 outputs).  The
// global loads of iteration t+1 are issued before the stages of iteration t.
//
// Boundary conditions: f^n ghost cells are loaded through the periodic wrap
// or the edge clamp, which is exactly the ghost fill of the scheme.  For a
// zero-gradient side, f^(1) ghost values must equal the edge cell's f^(1)
// (ghosts are refilled before every stage), so stage 2 redirects those
// reads to the clamped cell instead of using stage 1 evaluated at a ghost.
#pragma once

#include <hip/hip_runtime.h>

#include "cell.hpp"

namespace cdbm {

constexpr int FUSED_TX = 60;               // output columns per strip
constexpr int FUSED_R = 4;                 // rows per iteration
constexpr int FUSED_W0 = FUSED_TX + 8;     // F0 row width
constexpr int FUSED_W1 = FUSED_TX + 4;     // F1 row width (= 64 = one wave)
constexpr int FUSED_SLOTS = 2 * FUSED_R;   // ring depth
constexpr int FUSED_NT = FUSED_R * FUSED_W1;   // 256 threads

template <typename S>
__device__ __forceinline__ S coef_x(const KParams& K, int i, int z);
template <>
__device__ __forceinline__ float coef_x<float>(const KParams& K, int i, int z) { return K.cxf[i + z]; }
template <>
__device__ __forceinline__ double coef_x<double>(const KParams& K, int i, int z) { return K.cx[i + z]; }
template <typename S>
__device__ __forceinline__ S coef_y(const KParams& K, int i, int z);
template <>
__device__ __forceinline__ float coef_y<float>(const KParams& K, int i, int z) { return K.cyf[i + z]; }
template <>
__device__ __forceinline__ double coef_y<double>(const KParams& K, int i, int z) { return K.cy[i + z]; }

// Reads of one ring buffer around one cell.  Offsets are compile-time after
// unrolling; only one of (ox, oy) is ever nonzero.
template <typename S, int W>
struct RingLd {
    const S* ring;
    int slot[5];   // ring slot of rows offset -2..2
    int col[5];    // local column of columns offset -2..2
    __device__ __forceinline__ S operator()(int i, int ox, int oy) const {
        if (oy != 0) return ring[(slot[oy + 2] * NV + i) * W + col[2]];
        return ring[(slot[2] * NV + i) * W + col[ox + 2]];
    }
};

// One stage at one cell, f + dt L(f), with every run constant read from K at
// an opaque zero offset (see opaque_zero).
template <typename S, class Ld>
__device__ __forceinline__ void stage_cell_k(const Ld& ld, const KParams& K, S out[NV]) {
    const int z = opaque_zero();
    S f[NV];
    double fd[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        f[i] = ld(i, 0, 0);
        fd[i] = (double)f[i];
    }
    Parity g;
    to_parity(fd, g);
    const Macro m = macro_from_parity(g, K, (&K.inv_a)[z], z);
    double feq[NV];
    equilibrium(m, K, (&K.a)[z], feq, z);
    const double zr = (&K.z)[z];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        S adv = S(0);
        if (SX[i] > 0)
            adv = coef_x<S>(K, i, z) * nnd_pos<S>(ld(i, -2, 0), ld(i, -1, 0), f[i], ld(i, 1, 0));
        else if (SX[i] < 0)
            adv = coef_x<S>(K, i, z) * nnd_neg<S>(ld(i, -1, 0), f[i], ld(i, 1, 0), ld(i, 2, 0));
        if (SY[i] > 0)
            adv += coef_y<S>(K, i, z) * nnd_pos<S>(ld(i, 0, -2), ld(i, 0, -1), f[i], ld(i, 0, 1));
        else if (SY[i] < 0)
            adv += coef_y<S>(K, i, z) * nnd_neg<S>(ld(i, 0, -1), f[i], ld(i, 0, 1), ld(i, 0, 2));
        const S coll = (S)(zr * (fd[i] - feq[i]));
        out[i] = f[i] + (adv - coll);
    }
}

// Source row of a (possibly ghost) row index: periodic wrap or edge clamp.
// Uniform within a wave; cheap for the usual case of an offset below n.
__device__ __forceinline__ int source_row(int r, int n, int bc) {
    if (bc == CDBM_PERIODIC) {
        while (r < 0) r += n;
        while (r >= n) r -= n;
        return r;
    }
    return r < 0 ? 0 : (r >= n ? n - 1 : r);
}

__device__ __forceinline__ int map_index(int i, int n, int bc) { return wrap_or_clamp(i, n, bc); }

// Advance rows [ya, yb) of the strip starting at column x0 of one grid.
// All threads of the block must call this together (it synchronizes).
template <typename S>
__device__ __forceinline__ void fused_strip(const S* __restrict__ fin, S* __restrict__ fout,
                                            const KParams& K, int x0, int ya, int yb, S* F0,
                                            S* F1) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // 0..3, uniform
    const int nx = K.nx, ny = K.ny, bcx = K.bcx, bcy = K.bcy;
    const int64_t cells = (int64_t)nx * ny;

    // global columns this lane loads into F0 (lanes 0..63, plus 64..67 on lanes 0..3)
    const int gc_a = map_index(x0 - 4 + lane, nx, bcx);
    const int gc_b = map_index(x0 - 4 + 64 + (lane & 3), nx, bcx);

    // ring slot of a row: rows are >= ya - 4 - 2R when used
    const int yref0 = ya - 4 - FUSED_SLOTS;
    const int yref1 = ya - 2 - FUSED_SLOTS;
    auto slot0 = [&](int r) { return (r - yref0) & (FUSED_SLOTS - 1); };
    auto slot1 = [&](int r) { return (r - yref1) & (FUSED_SLOTS - 1); };

    const int nrows = yb - ya;
    const int niter = (nrows + FUSED_R - 1) / FUSED_R + 2;

    // each wave loads 16 of the 64 (row, velocity) lines of an iteration
    constexpr int LINES = FUSED_R * NV / 4;   // per wave
    S pre_a[LINES], pre_b[LINES];
    auto issue_loads = [&](int t) {
        const int rbase = ya - 4 + t * FUSED_R;
#pragma unroll
        for (int k = 0; k < LINES; ++k) {
            const int line = wave * LINES + k;       // 0..63
            const int rr = line / NV, i = line % NV;
            const int gr = source_row(rbase + rr, ny, bcy);
            const S* src = fin + (int64_t)i * cells + (int64_t)gr * nx;
            pre_a[k] = src[gc_a];
            pre_b[k] = (lane < 4) ? src[gc_b] : S(0);
        }
    };
    auto store_loads = [&](int t) {
        const int rbase = ya - 4 + t * FUSED_R;
#pragma unroll
        for (int k = 0; k < LINES; ++k) {
            const int line = wave * LINES + k;
            const int rr = line / NV, i = line % NV;
            S* dst = F0 + (slot0(rbase + rr) * NV + i) * FUSED_W0;
            dst[lane] = pre_a[k];
            if (lane < 4) dst[64 + lane] = pre_b[k];
        }
    };

    issue_loads(0);
    for (int t = 0; t < niter; ++t) {
        __syncthreads();   // previous stages are done with the slots being overwritten
        store_loads(t);
        if (t + 1 < niter) issue_loads(t + 1);
        __syncthreads();

        // stage 1: f^(1) at row r1, column x0 - 2 + lane
        if (t >= 1) {
            const int r1 = ya - 2 + (t - 1) * FUSED_R + wave;
            RingLd<S, FUSED_W0> ld;
            ld.ring = F0;
#pragma unroll
            for (int o = -2; o <= 2; ++o) {
                ld.slot[o + 2] = slot0(r1 + o);
                ld.col[o + 2] = lane + 2 + o;
            }
            S out[NV];
            stage_cell_k<S>(ld, K, out);
            S* dst = F1 + slot1(r1) * NV * FUSED_W1 + lane;
#pragma unroll
            for (int i = 0; i < NV; ++i) dst[i * FUSED_W1] = out[i];
        }
        __syncthreads();

        // stage 2: f^{n+1} at row r2, column x0 + lane
        if (t >= 2) {
            const int r2 = ya + (t - 2) * FUSED_R + wave;
            const int x = x0 + lane;
            const bool active = lane < FUSED_TX && x < nx && r2 < yb;
            RingLd<S, FUSED_W1> ld;
            ld.ring = F1;
#pragma unroll
            for (int o = -2; o <= 2; ++o) {
                const int rr = (bcy == CDBM_ZERO_GRADIENT) ? min(max(r2 + o, 0), ny - 1) : r2 + o;
                const int cc = (bcx == CDBM_ZERO_GRADIENT) ? min(max(x + o, 0), nx - 1) : x + o;
                ld.slot[o + 2] = slot1(rr);
                ld.col[o + 2] = min(max(cc - (x0 - 2), 0), FUSED_W1 - 1);
            }
            S out[NV];
            stage_cell_k<S>(ld, K, out);
            if (active) {
                const S* fn = F0 + slot0(r2) * NV * FUSED_W0 + lane + 4;
                S* dst = fout + (int64_t)r2 * nx + x;
#pragma unroll
                for (int i = 0; i < NV; ++i)
                    dst[(int64_t)i * cells] = S(0.5) * fn[i * FUSED_W0] + S(0.5) * out[i];
            }
        }
    }
    __syncthreads();
}

}  // namespace cdbm
