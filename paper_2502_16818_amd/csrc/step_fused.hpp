// Fused two-stage Runge-Kutta step of the CDBM (both stages in one pass
// over HBM).
//
// A block owns a strip of TX = 56 output columns and streams down the grid
// in y, R = 6 rows per iteration (one wave per row), keeping two ring
// buffers of R + 4 rows in LDS:
//   F0: f^n rows, TX + 8 = 64 columns (x halo of 4 each side);
//   F1: f^(1) = f^n + dt L(f^n) rows, TX + 4 = 60 columns at a stride of 64.
// In FP64 both rows are 512 bytes, so one base address and immediate
// offsets serve the LDS accesses of all 16 velocities of a cell, and the two
// rings fill the 160 KB of LDS.
// Iteration t (rows relative to the segment start):
//   load  f^n    rows [4 + (t-2)R, 4 + (t-1)R)   (global -> registers -> F0)
//   stage 1      rows [2 + (t-2)R, 2 + (t-1)R)   (F0 -> F1; one cell per thread)
//   stage 2      rows [(t-2)R, (t-1)R)           (F1, F0 -> f^{n+1} in HBM)
// Each stage runs just two rows behind what it needs, so R + 4 rows of each
// ring are live at once; each f value crosses HBM once in and once out per
// step, and stage 1 is recomputed only on the 2-column x halo (60 columns
// for 56 outputs).  The global loads of iteration t+1 are issued during
// iteration t, in two halves: before stage 1 and before stage 2.  This strip
// serves FP64 storage; FP32 storage uses the wider strip of step_wide.hpp.
//
// Boundary conditions: f^n ghost cells are loaded through the periodic wrap
// or the edge clamp, which is exactly the ghost fill of the scheme.  For a
// zero-gradient side, f^(1) ghost values must equal the edge cell's f^(1)
// (ghosts are refilled before every stage), so stage 2 redirects those
// reads to the clamped cell instead of using stage 1 evaluated at a ghost.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "cell.hpp"

namespace cdbm {

// Geometry of the strip: TX output columns; F0 rows hold TX + 8 columns of
// f^n (4 halo columns each side), F1 rows the TX + 4 columns of f^(1) that
// stage 2 reads; both rows are 64 elements (512 bytes in FP64), one column
// per lane.  R rows per iteration, one wave per row; ring depth R + 4.
// FP64: 56 outputs, 6 rows (384 threads, all 160 KB of LDS).  The wider
// 60-column strip with 4 rows (one wave per SIMD) left every LDS and barrier
// latency exposed and was 6 % slower.
template <typename S>
struct FusedGeom;
template <>
struct FusedGeom<double> {
    static constexpr int TX = 56;
    static constexpr int W0 = 64;
    static constexpr int W1 = 64;
    static constexpr int R = 6;
    static constexpr int SLOTS = R + 4;
    static constexpr int NT = R * 64;
    static constexpr int F0_ELEMS = SLOTS * NV * W0;
    static constexpr int F1_ELEMS = SLOTS * NV * W1;
    static_assert(W0 == TX + 8 && W1 >= TX + 4 && W1 <= 64, "one column per lane");
};

// NND coefficients -dt v_ir / dr of a stage: HALF selects the halved ones of
// the second Runge-Kutta stage.
template <typename S, bool HALF>
__device__ __forceinline__ S stage_coef_x(const KParams& K, int i, int z) {
    if constexpr (sizeof(S) == 4) return HALF ? K.cxhf[i + z] : K.cxf[i + z];
    else return HALF ? K.cxh[i + z] : K.cx[i + z];
}
template <typename S, bool HALF>
__device__ __forceinline__ S stage_coef_y(const KParams& K, int i, int z) {
    if constexpr (sizeof(S) == 4) return HALF ? K.cyhf[i + z] : K.cyf[i + z];
    else return HALF ? K.cyh[i + z] : K.cy[i + z];
}

// -z/2 (axis groups, grp 0) or -z/4 (diagonal groups, grp 1) of a stage.
template <typename S, bool HALF>
__device__ __forceinline__ S stage_relax(const KParams& K, int grp, int z) {
    if constexpr (sizeof(S) == 4) return K.nzqf[HALF][grp + z];
    else return K.nzq[HALF][grp + z];
}

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

// Makes v available at this point of the program.  Stores that only some
// lanes perform sit in a branch, and the compiler would otherwise move the
// arithmetic feeding them into that branch, apart from the lane shifts
// below, which must run in every lane.
__device__ __forceinline__ void materialize(float& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void materialize(double& v) { asm volatile("" : "+v"(v)); }

// Value of a 32-bit register in lane - 1 (from_left) or lane + 1
// (from_right) of the wave: DPP whole-wave shifts, which the compiler folds
// into the instruction that uses the value.  Lane 0 (from_left) and lane 63
// (from_right) receive 0.
__device__ __forceinline__ float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
// 64-bit values move as two 32-bit halves (two shifts).
template <int CTRL>
__device__ __forceinline__ double shift_lanes(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xf, 0xf, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double from_left(double v) { return shift_lanes<0x138>(v); }
__device__ __forceinline__ double from_right(double v) { return shift_lanes<0x130>(v); }

// One stage at one cell with every run constant read from K at an opaque
// zero offset (see opaque_zero).  First stage (HALF = false): returns
// f + dt L(f).  Second stage (HALF = true): returns (f + dt L(f)) / 2, with
// the 1/2 folded into the coefficients, so that the Heun combination is
// f^n / 2 plus the result.
//
// XLANE: the lanes of the wave hold consecutive cells of a row,
// and the x-direction NND takes the minmod of the neighbouring cell from the
// neighbouring lane.  Each lane forms M = minmod(f_{j+1} - f_j, f_j - f_{j-1});
// the positive-velocity difference needs M of lane j - 1 and the negative one
// M of lane j + 1, so lanes 0 and 63 return garbage and the caller discards
// them.  The arithmetic is the same as nnd_pos / nnd_neg term by term, so the
// results are bitwise those of the per-lane form.  All 64 lanes must run it.
template <typename S, bool HALF, class Ld, bool XLANE = false>
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
    double neq[NV];
    nonequilibrium(g, m, K, (&K.a)[z], neq, z);
    // -z / k of the stage, k = 2 (axis groups) or 4 (diagonal groups)
    const S nza = stage_relax<S, HALF>(K, 0, z), nzd = stage_relax<S, HALF>(K, 1, z);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        S adv = S(0);
        if constexpr (XLANE) {
            if (SX[i] != 0) {
                const S dl = f[i] - ld(i, -1, 0), dr = ld(i, 1, 0) - f[i];
                const S M = minmod(dr, dl);
                const S cx = stage_coef_x<S, HALF>(K, i, z);
                if (SX[i] > 0) adv = cx * (dl + S(0.5) * (M - from_left(M)));
                else adv = cx * (dr - S(0.5) * (from_right(M) - M));
            }
        } else if (SX[i] > 0)
            adv = stage_coef_x<S, HALF>(K, i, z) *
                  nnd_pos<S>(ld(i, -2, 0), ld(i, -1, 0), f[i], ld(i, 1, 0));
        else if (SX[i] < 0)
            adv = stage_coef_x<S, HALF>(K, i, z) *
                  nnd_neg<S>(ld(i, -1, 0), f[i], ld(i, 1, 0), ld(i, 2, 0));
        if (SY[i] > 0)
            adv += stage_coef_y<S, HALF>(K, i, z) *
                   nnd_pos<S>(ld(i, 0, -2), ld(i, 0, -1), f[i], ld(i, 0, 1));
        else if (SY[i] < 0)
            adv += stage_coef_y<S, HALF>(K, i, z) *
                   nnd_neg<S>(ld(i, 0, -1), f[i], ld(i, 0, 1), ld(i, 0, 2));
        const S d = fma((i & 4) ? nzd : nza, (S)neq[i], adv);
        out[i] = HALF ? fma(S(0.5), f[i], d) : f[i] + d;
    }
}

// Block barrier that orders LDS traffic only.  The waves of a block share
// data through LDS alone (f^n is read-only, each f^{n+1} element is written
// by one thread), so global loads and stores may stay in flight across it;
// __syncthreads() would also drain them at every barrier.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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

// 16-byte vector of the storage type (4 floats or 2 doubles).
template <typename S>
struct Chunk;
template <>
struct Chunk<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Chunk<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};

// Stores the 16 velocities of one cell, v[i] at byte offset xo + i * plane
// from `row`, through a raw buffer descriptor: the row start and the plane
// offsets are wave-uniform (scalar registers) and the column offset xo is the
// only vector operand, so the stores take no per-velocity address
// arithmetic on the vector unit.  `row` must be wave-uniform and every offset
// below 2^32, which the chunked form guarantees (at most 4 GiB per grid).
// Word 3 of the descriptor is the 32-bit data format of the gfx9 family.
// (Used by the FP64 strip: in the FP32 strips the same stores measured
// slightly slower than 64-bit addresses.)
__device__ __forceinline__ void store_planes(double* row, uint32_t plane, uint32_t xo,
                                             const double v[NV]) {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(row, 0, -1, 0x00020000);
    // plane offsets formed here, one scalar add each: hoisted out of the
    // caller's loop they would take 16 scalar registers for its whole length
    const uint32_t step = plane + (uint32_t)opaque_zero();
    uint32_t so = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v[i]), rs, (int)xo, (int)so,
                                              0);
        so += step;
    }
}

// Elements per 16-byte chunk of the chunked form.
template <typename S>
constexpr int fused_chunk_elems() {
    return 16 / (int)sizeof(S);
}
inline bool aligned16(const void* a, const void* b) {
    return (((uintptr_t)a | (uintptr_t)b) & 15) == 0;
}
// Can a grid of nx * ny cells between these buffers use the chunked form?
// Besides the chunk geometry, the whole f buffer must be addressable with
// 32-bit byte offsets from a row start.
template <typename S>
inline bool fused_chunked(int nx, int ny, const void* fin, const void* fout) {
    return nx % fused_chunk_elems<S>() == 0 && aligned16(fin, fout) &&
           (uint64_t)NV * (uint64_t)nx * (uint64_t)ny * sizeof(S) <= (uint64_t(1) << 32);
}

// Advance rows [ya, yb) of the strip starting at column x0 of one grid.
// All threads of the block must call this together (it synchronizes).
//
// VEC = false: every lane moves one column of each row (any grid).
// VEC = true: rows move between HBM and LDS in 16-byte chunks spread over
// the lanes of the wave; needs nx to be a multiple of the chunk width,
// 16-byte aligned buffers and 32-bit offsets (fused_chunked), so that every
// chunk of loaded columns lies inside one row.  Each lane keeps the byte
// offsets of its chunks from a row start for the whole strip.  A chunk left
// or right of the grid takes its periodic image; on a zero-gradient side
// those ghost columns are never read, because both stages redirect
// ghost-column reads to the edge column.  Every lane stores its own stage-2
// cell.
template <typename S, bool VEC>
__device__ __forceinline__ void fused_strip(const S* __restrict__ fin, S* __restrict__ fout,
                                            const KParams& K, int x0, int ya, int yb, S* F0,
                                            S* F1) {
    using G = FusedGeom<S>;
    using V = typename Chunk<S>::type;
    constexpr int R = G::R;
    constexpr int SLOTS = G::SLOTS;
    constexpr int TX = G::TX, W0 = G::W0, W1 = G::W1;
    constexpr int CW = 16 / (int)sizeof(S);        // elements per chunk
    constexpr int LCH = W0 / CW;                   // chunks per loaded velocity row
    constexpr int NLD = (NV * LCH + 63) / 64;      // chunk loads per lane and row
    static_assert(W0 % CW == 0 && TX % CW == 0 && 4 % CW == 0, "chunk geometry");
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // 0..R-1, uniform
    // Column of this lane in the stage windows: the x-direction NND shares
    // minmod terms between neighbouring lanes (stage_cell_k with XLANE), so
    // lane 0 and lane 63 only serve their neighbours; lane l computes column
    // l - 1 and lanes 1 .. 62 are kept (60 stage-1 and 56 stage-2 columns
    // are needed).
    const int ccol = lane - 1;
    const bool keep = lane >= 1 && lane <= 62;
    const int nx = K.nx, ny = K.ny, bcx = K.bcx, bcy = K.bcy;
    const int64_t cells = (int64_t)nx * ny;
    const int nrows = yb - ya;

    // ring slot of a row given relative to ya (rows >= -4 - R are ever used)
    auto slot = [&](int q) { return (q + 4 * SLOTS) % SLOTS; };

    // Chunk c = k * 64 + lane of a row: velocity c / per_row, chunk c % per_row.
    // Lanes past the last chunk repeat it (the same value to the same place).
    // ld_off: byte offsets of the chunks this lane loads, from the start of a
    // row of velocity 0.  A chunk left or right of the grid takes its
    // periodic image.
    uint32_t ld_off[VEC ? NLD : 1];
    if constexpr (VEC) {
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int c = min(k * 64 + lane, NV * LCH - 1);
            const int i = c / LCH, j = c - i * LCH;
            int cs = x0 - 4 + j * CW;
            if (cs < 0 || cs >= nx) {
                cs %= nx;
                if (cs < 0) cs += nx;
            }
            ld_off[k] = (uint32_t)(((int64_t)i * cells + cs) * (int64_t)sizeof(S));
        }
    }

    // wave w loads row 4 + (t-2)R + w (all 16 velocities) at iteration t;
    // only rows -4 .. nrows+3 are needed
    constexpr int NPRE = VEC ? NLD : NV;
    using P = typename std::conditional<VEC, V, S>::type;
    P pre[NPRE];
    // per-column form: the global column this lane loads into F0
    const int gc_a = VEC ? 0 : map_index(x0 - 4 + lane, nx, bcx);
    auto load_row = [&](int t) { return 4 + (t - 2) * R + wave; };
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
                if ((k < (NLD + 1) / 2 ? 0 : 1) == half) pre[k] = *(const V*)(base + ld_off[k]);
        } else {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                if ((i < NV / 2 ? 0 : 1) != half) continue;
                pre[i] = src[(int64_t)i * cells + gc_a];
            }
        }
    };
    auto store_loads = [&](int t) {
        const int q = load_row(t);
        if (!wanted(q)) return;
        S* dst = F0 + slot(q) * NV * W0;
        if constexpr (VEC) {
            // chunk c sits at element c * CW of the slot (W0 = LCH * CW)
#pragma unroll
            for (int k = 0; k < NLD; ++k)
                *(V*)(dst + min(k * 64 + lane, NV * LCH - 1) * CW) = pre[k];
        } else {
#pragma unroll
            for (int i = 0; i < NV; ++i) dst[i * W0 + lane] = pre[i];
        }
    };

    // first iteration whose loads reach row -4; stage 2 finishes at t_end
    const int t0 = 2 - (8 + R - 1) / R;
    const int t_end = (nrows + R - 1) / R + 1;
    issue_loads(t0, 0);
    issue_loads(t0, 1);
    for (int t = t0; t <= t_end; ++t) {
        lds_barrier();   // the stages of iteration t-1 are done with the slots reused below
        store_loads(t);
        if (t < t_end) issue_loads(t + 1, 0);
        lds_barrier();

        // stage 1: f^(1) at row q1, column x0 - 2 + ccol
        const int q1 = 2 + (t - 2) * R + wave;
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
        }
        lds_barrier();

        if (t < t_end) issue_loads(t + 1, 1);
        // stage 2: f^{n+1} at row q2, column x0 + ccol
        const int q2 = (t - 2) * R + wave;
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
                const S* fn = F0 + slot(q2) * NV * W0 + 4 + ccol;   // f^n of the cell
#pragma unroll
                for (int i = 0; i < NV; ++i) out[i] = fma(S(0.5), fn[i * W0], out[i]);
                if constexpr (VEC) {
                    store_planes(fout + (int64_t)r2 * nx, (uint32_t)(cells * (int64_t)sizeof(S)),
                                 (uint32_t)x * (uint32_t)sizeof(S), out);
                } else {
                    S* dst = fout + (int64_t)r2 * nx + x;
#pragma unroll
                    for (int i = 0; i < NV; ++i) dst[(int64_t)i * cells] = out[i];
                }
            }
        }
    }
    lds_barrier();
}

}  // namespace cdbm
