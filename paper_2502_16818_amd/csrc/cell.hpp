// Per-cell device arithmetic of the CDBM step, shared by every kernel.
//
// Equilibrium (Eqs. (4)-(7)).  For a cell with distributions f_i:
//   1. parity combinations g of each group of four f_i (sums and differences
//      of opposite velocities);
//   2. conserved moments rho, j, 2E from g, then u = j / rho and
//      T = (2E / rho - |u|^2) / (D + I)   (energy row of Eq. (4));
//   3. raw Maxwellian moments m^eq / rho in the parity blocks (the exact
//      central-to-raw shift of the central moments of Eq. (5));
//   4. h = rho * Binv m-hat per block, with the block inverses of the moment
//      matrix at u = 0 (built on the host; rows pre-scaled by 1/2 or 1/4);
//   5. unpack h into the 16 f_i^eq with additions.
// All of it runs in double, in every precision mode.
//
// NND (Eqs. (12)-(20)).  For a velocity component v > 0 only f^+ = v f is
// nonzero and the flux difference H(j+1/2) - H(j-1/2) reduces to
//   v [ (f_j - f_{j-1}) + (minmod(f_{j+1}-f_j, f_j-f_{j-1})
//                          - minmod(f_j-f_{j-1}, f_{j-1}-f_{j-2})) / 2 ],
// and for v < 0 (only f^- nonzero) to the mirror image
//   v [ (f_{j+1} - f_j) - (minmod(f_{j+2}-f_{j+1}, f_{j+1}-f_j)
//                          - minmod(f_{j+1}-f_j, f_j-f_{j-1})) / 2 ].
// minmod of Eq. (16) equals the median of (X, Y, 0).
#pragma once

#include <hip/hip_runtime.h>

#include "model.hpp"

namespace cdbm {

__device__ __forceinline__ float minmod(float X, float Y) {
    return __builtin_amdgcn_fmed3f(X, Y, 0.0f);
}
__device__ __forceinline__ double minmod(double X, double Y) {
    return fmax(fmin(X, Y), fmin(fmax(X, Y), 0.0));
}

// D for a positive component (stencil j-2 .. j+1) and a negative one (j-1 .. j+2).
template <typename R>
__device__ __forceinline__ R nnd_pos(R m2, R m1, R c0, R p1) {
    const R d0 = c0 - m1;
    return d0 + R(0.5) * (minmod(p1 - c0, d0) - minmod(d0, m1 - m2));
}
template <typename R>
__device__ __forceinline__ R nnd_neg(R m1, R c0, R p1, R p2) {
    const R d1 = p1 - c0;
    return d1 - R(0.5) * (minmod(p2 - p1, d1) - minmod(d1, c0 - m1));
}

struct Parity {
    double ee[6], oe[4], eo[4], oo[2];
};

// Parity combinations of the 16 distributions (velocity order of model.hpp).
__device__ __forceinline__ void to_parity(const double f[NV], Parity& g) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int a = 8 * q;       // axis group (a or c)
        const int d = 8 * q + 4;   // diagonal group (b or d)
        g.ee[3 * q + 0] = f[a + 0] + f[a + 2];
        g.ee[3 * q + 1] = f[a + 1] + f[a + 3];
        g.oe[2 * q + 0] = f[a + 0] - f[a + 2];
        g.eo[2 * q + 0] = f[a + 1] - f[a + 3];
        const double s01 = f[d + 0] + f[d + 1], s23 = f[d + 2] + f[d + 3];
        const double d01 = f[d + 0] - f[d + 1], d23 = f[d + 2] - f[d + 3];
        g.ee[3 * q + 2] = s01 + s23;
        g.oe[2 * q + 1] = d01 - d23;
        g.eo[2 * q + 1] = s01 - s23;
        g.oo[q] = d01 + d23;
    }
}

struct Macro {
    double rho, ux, uy, T;
};

// `inv_a` = 1 / (D + I).  `z` is a zero offset for the constant-table reads;
// kernels pass an opaque zero so the compiler reloads the tables where they
// are used instead of holding them in scalar registers across loops.
__device__ __forceinline__ Macro macro_from_parity(const Parity& g, const KParams& K, double inv_a,
                                                   int z = 0) {
    const double rho = ((g.ee[0] + g.ee[1]) + (g.ee[2] + g.ee[3])) + (g.ee[4] + g.ee[5]);
    double jx = 0.0, jy = 0.0, e2 = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        jx = fma(K.jx[c + z], g.oe[c], jx);
        jy = fma(K.jy[c + z], g.eo[c], jy);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) e2 = fma(K.en[c + z], g.ee[c], e2);
    // 1 / rho: hardware reciprocal refined by two Newton steps (error ~1 ulp)
    double inv = __builtin_amdgcn_rcp(rho);
    inv = fma(inv, fma(-rho, inv, 1.0), inv);
    inv = fma(inv, fma(-rho, inv, 1.0), inv);
    Macro m;
    m.rho = rho;
    m.ux = jx * inv;
    m.uy = jy * inv;
    m.T = (e2 * inv - (m.ux * m.ux + m.uy * m.uy)) * inv_a;
    return m;
}

// f^eq of the state m (Eq. (7)), through the raw moments and the shared
// parity-block inverses; a = D + I.
__device__ __forceinline__ void equilibrium(const Macro& m, const KParams& K, double a,
                                            double feq[NV], int z = 0) {
    const double ux = m.ux, uy = m.uy, T = m.T;
    const double ux2 = ux * ux, uy2 = uy * uy, u2 = ux2 + uy2, uxy = ux * uy;
    const double aT = a * T;
    const double A2 = u2 + aT + 2.0 * T;   // u^2 + (D+I+2) T
    const double A4 = A2 + 2.0 * T;        // u^2 + (D+I+4) T
    // raw moments / rho, rows (1,4,5,7,14,16), (2,8,10,12), (3,9,11,13), (6,15)
    const double mee[6] = {1.0, u2 + aT, ux2 + T, uy2 + T, ux2 * A4 + T * A2, uy2 * A4 + T * A2};
    const double moe[4] = {ux, ux * A2, ux * (ux2 + 3.0 * T), ux * (uy2 + T)};
    const double meo[4] = {uy, uy * A2, uy * (ux2 + T), uy * (uy2 + 3.0 * T)};
    const double moo[2] = {uxy, uxy * A4};
    double hee[6], hoe[4], heo[4], hoo[2];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        double s = K.iee[r][z];
#pragma unroll
        for (int c = 1; c < 6; ++c) s = fma(K.iee[r][c + z], mee[c], s);
        hee[r] = m.rho * s;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double so = 0.0, se = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            so = fma(K.ioe[r][c + z], moe[c], so);
            se = fma(K.ieo[r][c + z], meo[c], se);
        }
        hoe[r] = m.rho * so;
        heo[r] = m.rho * se;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
        hoo[r] = m.rho * fma(K.ioo[r][z], moo[0], K.ioo[r][1 + z] * moo[1]);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int a = 8 * q, d = 8 * q + 4;
        feq[a + 0] = hee[3 * q + 0] + hoe[2 * q];
        feq[a + 2] = hee[3 * q + 0] - hoe[2 * q];
        feq[a + 1] = hee[3 * q + 1] + heo[2 * q];
        feq[a + 3] = hee[3 * q + 1] - heo[2 * q];
        const double p = hee[3 * q + 2] + heo[2 * q + 1], n = hee[3 * q + 2] - heo[2 * q + 1];
        const double r = hoe[2 * q + 1] + hoo[q], s = hoe[2 * q + 1] - hoo[q];
        feq[d + 0] = p + r;
        feq[d + 1] = p - r;
        feq[d + 2] = n - s;
        feq[d + 3] = n + s;
    }
}

// k (f - f^eq) for the 16 velocities, k = 2 for the axis groups and 4 for
// the diagonal ones, formed in the parity basis: with g the parity
// combinations of f and B m-hat the (row-scaled by 1/k) block contraction,
// the parity combinations of k (f - f^eq) are g_r - k rho (B m-hat)_r, and
// unpacking them (additions only) gives k (f_i - f_i^eq).
__device__ __forceinline__ void nonequilibrium(const Parity& g, const Macro& m, const KParams& K,
                                               double a, double out[NV], int z = 0) {
    const double ux = m.ux, uy = m.uy, T = m.T;
    const double ux2 = ux * ux, uy2 = uy * uy, u2 = ux2 + uy2, uxy = ux * uy;
    const double aT = a * T;
    const double A2 = u2 + aT + 2.0 * T;
    const double A4 = A2 + 2.0 * T;
    const double mee[6] = {1.0, u2 + aT, ux2 + T, uy2 + T, ux2 * A4 + T * A2, uy2 * A4 + T * A2};
    const double moe[4] = {ux, ux * A2, ux * (ux2 + 3.0 * T), ux * (uy2 + T)};
    const double meo[4] = {uy, uy * A2, uy * (ux2 + T), uy * (uy2 + 3.0 * T)};
    const double moo[2] = {uxy, uxy * A4};
    const double n2 = -2.0 * m.rho, n4 = -4.0 * m.rho;
    // group of each parity component (k = 2 for a and c, 4 for b and d):
    // ee (a, a, b, c, c, d), oe/eo (a, b, c, d), oo (b, d)
    double tee[6], toe[4], teo[4], too[2];
    // even-even block in mirror form (KParams::eep, ees): the rows of a
    // mirrored pair of unknowns share their part even in x <-> y, and the
    // constant term (mee[0] = 1) goes onto g first
    const double s23 = mee[2] + mee[3], d23 = mee[2] - mee[3];
    const double s45 = mee[4] + mee[5], d45 = mee[4] - mee[5];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r0 = 3 * q;   // pair (r0, r0 + 1), axis groups: n2
        const double P =
            fma(K.eep[q][3 + z], s45, fma(K.eep[q][2 + z], s23, K.eep[q][1 + z] * mee[1]));
        const double Q = fma(K.eep[q][5 + z], d45, K.eep[q][4 + z] * d23);
        tee[r0] = fma(n2, P + Q, fma(n2, K.eep[q][z], g.ee[r0]));
        tee[r0 + 1] = fma(n2, P - Q, fma(n2, K.eep[q][z], g.ee[r0 + 1]));
        const int rd = 3 * q + 2;   // diagonal groups: n4
        const double D =
            fma(K.ees[q][3 + z], s45, fma(K.ees[q][2 + z], s23, K.ees[q][1 + z] * mee[1]));
        tee[rd] = fma(n4, D, fma(n4, K.ees[q][z], g.ee[rd]));
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double so = 0.0, se = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            so = fma(K.ioe[r][c + z], moe[c], so);
            se = fma(K.ieo[r][c + z], meo[c], se);
        }
        const double n = (r & 1) ? n4 : n2;
        toe[r] = fma(n, so, g.oe[r]);
        teo[r] = fma(n, se, g.eo[r]);
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
        too[r] = fma(n4, fma(K.ioo[r][z], moo[0], K.ioo[r][1 + z] * moo[1]), g.oo[r]);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int a0 = 8 * q, d0 = 8 * q + 4;
        out[a0 + 0] = tee[3 * q + 0] + toe[2 * q];
        out[a0 + 2] = tee[3 * q + 0] - toe[2 * q];
        out[a0 + 1] = tee[3 * q + 1] + teo[2 * q];
        out[a0 + 3] = tee[3 * q + 1] - teo[2 * q];
        const double p = tee[3 * q + 2] + teo[2 * q + 1], n = tee[3 * q + 2] - teo[2 * q + 1];
        const double r = toe[2 * q + 1] + too[q], s = toe[2 * q + 1] - too[q];
        out[d0 + 0] = p + r;
        out[d0 + 1] = p - r;
        out[d0 + 2] = n - s;
        out[d0 + 3] = n + s;
    }
}

// A zero the compiler cannot see through (a scalar register set by an empty
// instruction sequence), re-created wherever constant tables are read.
__device__ __forceinline__ int opaque_zero() {
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return z;
}

// Boundary index map for a neighbour offset: periodic wrap or clamp.
__device__ __forceinline__ int wrap_or_clamp(int i, int n, int bc) {
    if (bc == CDBM_PERIODIC) {
        i %= n;
        return i < 0 ? i + n : i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

}  // namespace cdbm
