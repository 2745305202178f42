// Two time steps per pass over HBM (temporal blocking), FP32 storage.
//
// A block streams down a strip of TX = 48 output columns, R = 6 rows per
// iteration, two waves per row, and carries four rows of stages in LDS rings:
//   F0: f^n           (read from HBM)
//   F1: f^(1)   = f^n + dt L(f^n)                      stage 1 of step n
//   F2: f^{n+1} = f^n / 2 + (f^(1) + dt L(f^(1))) / 2  stage 2 of step n
//   F3: f^(1')  = f^{n+1} + dt L(f^{n+1})              stage 1 of step n + 1
// and writes f^{n+2} = f^{n+1} / 2 + (f^(1') + dt L(f^(1'))) / 2 to HBM: each
// f value crosses HBM once in and once out per two steps.  Every ring row
// holds strip columns -8 .. 55 (one per lane, lane l at column l - 8, rows
// of 64 floats, so all four rings fill the 160 KiB of LDS at R + 4 = 10 slots
// each); stage k is valid on columns -8 + 2k .. 55 - 2k, and the output on
// 0 .. 47.  Each stage takes the x-direction minmod terms of the
// neighbouring cells from the neighbouring lanes (stage_cell_k with XLANE),
// with the same per-cell arithmetic as the one-step kernels, so two steps
// here equal two single steps bit for bit.
//
// Iteration t, rows relative to the segment start, row r of the iteration
// (waves 2r and 2r + 1, which share the row's f^n loads):
//   phase A: wave 2r: stage 1 at row a = tR + r - 10 (F0 -> F1);
//            wave 2r + 1: stage 3 at row c = a - R - 4 (F2 -> F3);
//            the Heun terms f^n (F0, row a - 2) and f^{n+1} (F2, row c - 2)
//            of phase B's cells go to registers, because phase B refills or
//            rewrites those slots;
//   phase B: the f^n rows of the next iteration (loads issued a phase
//            ahead); wave 2r: stage 2 at row a - 2 (F1 -> F2); wave 2r + 1:
//            stage 4 at row c - 2 (F3 -> HBM).
// Two barriers per iteration; every wave runs one stage per phase, so the
// four SIMDs carry three waves and equal work each.  Zero-gradient sides: every stage redirects
// reads of ghost rows or columns to the edge cell, which equals the ghost
// refill of the scheme at that stage.
#pragma once

#include "step_fused.hpp"

namespace cdbm {

struct TwoStepGeom {
    static constexpr int TX = 48;       // output columns per strip
    static constexpr int HALO = 8;      // columns each side (4 stages x 2)
    static constexpr int W = 64;        // ring row (floats), one column per lane
    static constexpr int R = 6;         // rows per iteration, two waves each
    static constexpr int SLOTS = R + 4;
    static constexpr int NT = 2 * R * 64;
    static constexpr int RING_ELEMS = SLOTS * NV * W;
    static_assert(TX + 2 * HALO == W, "one column per lane");
};

// Advance rows [ya, yb) of the strip starting at column x0 by two steps.
// F: the four rings, each TwoStepGeom::RING_ELEMS floats.  All threads of
// the block call this together.  VEC: the 16-byte-chunk form
// (fused_chunked<float> must hold).
template <bool VEC>
__device__ __forceinline__ void fused_strip_2(const float* __restrict__ fin,
                                              float* __restrict__ fout, const KParams& K, int x0,
                                              int ya, int yb, float* F0, float* F1, float* F2,
                                              float* F3) {
    using S = float;
    using V = Chunk<float>::type;
    using G = TwoStepGeom;
    constexpr int R = G::R, SLOTS = G::SLOTS, W = G::W, HALO = G::HALO;
    constexpr int NLD = NV * W / 4 / 128;   // 16-byte chunks per lane and row: 2
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rw = wave >> 1;     // row of the iteration
    const int role = wave & 1;    // 0: stages 1 and 2; 1: stages 3 and 4
    const int ccol = lane - HALO;                              // strip column of this lane
    const int nx = K.nx, ny = K.ny, bcx = K.bcx, bcy = K.bcy;
    const int64_t cells = (int64_t)nx * ny;
    const int nrows = yb - ya;

    auto slot = [&](int q) { return (q + 8 * SLOTS) % SLOTS; };

    // Chunk c = 128k + 64 role + lane of a row: velocity c / 16 =
    // 8k + 4 role + lane / 16, columns x0 - 8 + 4 (lane % 16) ..; it lands at
    // element 4c of the F0 slot, and one per-lane byte offset serves every k.
    const uint32_t plane = (uint32_t)(cells * (int64_t)sizeof(S));
    uint32_t ld_lane = 0;
    if constexpr (VEC) {
        int cs = x0 - HALO + 4 * (lane & 15);
        if (cs < 0 || cs >= nx) {   // periodic image (zero-gradient ghosts are never read)
            cs %= nx;
            if (cs < 0) cs += nx;
        }
        ld_lane = (uint32_t)(lane >> 4) * plane + (uint32_t)cs * (uint32_t)sizeof(S);
    }
    const int gc = VEC ? 0 : map_index(x0 + ccol, nx, bcx);

    constexpr int NPRE = VEC ? NLD : NV / 2;
    using P = typename std::conditional<VEC, V, S>::type;
    P pre[NPRE];
    auto load_row = [&](int t) { return t * R + rw - 8; };
    auto wanted = [&](int q) { return q >= -8 && q < nrows + 8; };
    auto issue_loads = [&](int t, int half) {
        const int q = load_row(t);
        if (!wanted(q)) return;
        const S* src = fin + (int64_t)source_row(ya + q, ny, bcy) * nx;
        if constexpr (VEC) {
            const char* base = (const char*)src;
#pragma unroll
            for (int k = 0; k < NLD; ++k)
                if (k == half)
                    pre[k] = *(const V*)(base + (uint32_t)(8 * k + 4 * role) * plane + ld_lane);
        } else {
            // wave 2r moves velocities 0 .. 7, wave 2r + 1 velocities 8 .. 15
#pragma unroll
            for (int i = 0; i < NV / 2; ++i)
                if (i / (NV / 4) == half) pre[i] = src[(int64_t)(i + 8 * role) * cells + gc];
        }
    };
    auto store_loads = [&](int t) {
        const int q = load_row(t);
        if (!wanted(q)) return;
        S* dst = F0 + slot(q) * NV * W;
        if constexpr (VEC) {
#pragma unroll
            for (int k = 0; k < NLD; ++k) *(V*)(dst + 4 * (128 * k + 64 * role + lane)) = pre[k];
        } else {
#pragma unroll
            for (int i = 0; i < NV / 2; ++i) dst[(i + 8 * role) * W + lane] = pre[i];
        }
    };
    // reads of ring `ring` around (row q, strip column ccol); ghost rows and
    // columns of a zero-gradient side go to the edge cell
    auto ring_ld = [&](const S* ring, int q) {
        RingLd<S, W> ld;
        ld.ring = ring;
        const int r = ya + q;
        const int x = x0 + ccol;
#pragma unroll
        for (int o = -2; o <= 2; ++o) {
            const int rr = (bcy == CDBM_ZERO_GRADIENT) ? min(max(r + o, 0), ny - 1) : r + o;
            const int cc = (bcx == CDBM_ZERO_GRADIENT) ? min(max(x + o, 0), nx - 1) : x + o;
            ld.slot[o + 2] = slot(rr - ya);
            ld.col[o + 2] = min(max(cc - (x0 - HALO), 0), W - 1);   // discarded lanes read in bounds
        }
        return ld;
    };

    // First and last iteration: loads reach row -8 at t = 0; the last
    // output row nrows - 1 is stage 4's row (t - 1) R + r - 16.
    const int t0 = 0;
    const int t_end = (nrows + 15) / R + 1;
    issue_loads(t0, 0);
    issue_loads(t0, 1);
    store_loads(t0);
    issue_loads(t0 + 1, 0);
    lds_barrier();   // the previous segment of this block is done with the rings
    S fnh[NV];   // Heun term of this lane's phase-B cell
    for (int t = t0; t <= t_end; ++t) {
        if (t < t_end) issue_loads(t + 1, 1);
        const int a = t * R + rw - 10;   // stage 1 row
        const int b = a - 2;             // stage 2 row
        const int c = a - R - 4;         // stage 3 row
        const int d = c - 2;             // stage 4 row
        // phase A: stage 1 (role 0) or stage 3 (role 1), and the Heun term
        // of phase B's cell
        const int qa = role ? c : a;
        const int qb = role ? d : b;
        const int ha = role ? 2 : 6;   // stage rows needed: [-ha, nrows + ha)
        const int hb = role ? 0 : 4;
        if (qa >= -ha && qa < nrows + ha) {
            S out[NV];
            stage_cell_k<S, false, RingLd<S, W>, true>(ring_ld(role ? F2 : F0, qa), K, out);
            S* dst = (role ? F3 : F1) + slot(qa) * NV * W + lane;
#pragma unroll
            for (int i = 0; i < NV; ++i) dst[i * W] = out[i];
        }
        if (qb >= -hb && qb < nrows + hb) {
            const S* src = (role ? F2 : F0) + slot(qb) * NV * W + lane;
#pragma unroll
            for (int i = 0; i < NV; ++i) fnh[i] = src[i * W];
        }
        lds_barrier();

        // phase B
        if (t < t_end) {
            store_loads(t + 1);
            if (t + 1 < t_end) issue_loads(t + 2, 0);
        }
        // stage 2 (role 0, into F2) or stage 4 (role 1, to HBM)
        if (qb >= -hb && qb < nrows + hb) {
            S out[NV];
            stage_cell_k<S, true, RingLd<S, W>, true>(ring_ld(role ? F3 : F1, qb), K, out);
#pragma unroll
            for (int i = 0; i < NV; ++i) materialize(out[i]);   // every lane runs the lane shifts
            if (role == 0) {
                S* dst = F2 + slot(qb) * NV * W + lane;
#pragma unroll
                for (int i = 0; i < NV; ++i) dst[i * W] = fma(S(0.5), fnh[i], out[i]);
            } else {
                const int x = x0 + ccol;
                if (lane >= HALO && lane < HALO + G::TX && x < nx) {
                    S* dst = fout + (int64_t)(ya + qb) * nx + x;
#pragma unroll
                    for (int i = 0; i < NV; ++i)
                        dst[(int64_t)i * cells] = fma(S(0.5), fnh[i], out[i]);
                }
            }
        }
        lds_barrier();   // the next phase A overwrites slots read above
    }
}

}  // namespace cdbm
