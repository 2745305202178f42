// Reverse-mode (transpose) arithmetic of one Runge-Kutta stage of the CDBM.
//
// A stage is E(g) = g + dt L(g) with L(g)_i = c_x D_x(g_i) + c_y D_y(g_i)
// - (g_i - g_i^eq) / tau (c = -dt v_ir / dr, D the NND flux difference of
// Eqs. (12)-(20)).  Its transpose applied to a vector a at cell y is
//   a_i + dt (J_adv^T a)_i - (dt/tau) (a_i - [(d g^eq / d g)^T a]_i).
//
// NND transpose.  With the minmod selections fixed, D is linear.  The face
// selection s(x) = (alpha, beta) of minmod(d(x+1/2), d(x-1/2)) (alpha: the
// first argument is taken, beta: the second, neither: 0) follows the branch
// order of Eq. (16): zero if the differences do not share a strict sign,
// else the first argument when |X| <= |Y|.  For v > 0
//   D(x) = d(x-1/2) + (mm(x) - mm(x-1)) / 2,  mm(x) = minmod(d(x+1/2), d(x-1/2)),
// so dD(x)/df(x+k) for k = +1, 0, -1, -2 is
//   a(x)/2,  1 + (b(x) - a(x-1) - a(x))/2,  -1 - (b(x) - a(x-1) + b(x-1))/2,  b(x-1)/2
// and for v < 0, D(x) = d(x+1/2) - (mm(x+1) - mm(x)) / 2 gives for k = +2..-1
//   -a(x+1)/2,  1 + (a(x+1) - b(x+1) + a(x))/2,  -1 + (b(x+1) - a(x) + b(x))/2,  -b(x)/2.
// The transpose gathers, at an extended position p, sum_k coef_k(p-k) a(p-k)
// over real cells p-k.  Ghost positions of a zero-gradient side alias the
// edge cell, so their gathers are added to it; periodic positions wrap.
//
// Equilibrium transpose.  f^eq = P h with h = rho B mhat(u, T) (P: unpacking
// of parity combinations, B: scaled block inverses).  P^T is the parity
// transform itself, so with w = B^T P^T a:
//   g_rho = w . mhat,  g_q = rho w . d mhat / d q  (q = u_x, u_y, T),
// and [(d f^eq/d g)^T a]_k = g_rho + (g_ux (v_kx - u_x) + g_uy (v_ky - u_y)
//   + g_T (|v_k - u|^2 + eta_k^2 - (D+I) T) / (D+I)) / rho.
#pragma once

#include <hip/hip_runtime.h>

#include "cell.hpp"

namespace cdbm {

// Parity form h of f^eq (f^eq = unpacking of h, see equilibrium()).
__device__ __forceinline__ void equilibrium_parity(const Macro& m, const KParams& K, double a,
                                                   Parity& h) {
    const double ux = m.ux, uy = m.uy, T = m.T;
    const double ux2 = ux * ux, uy2 = uy * uy, u2 = ux2 + uy2, uxy = ux * uy;
    const double aT = a * T;
    const double A2 = u2 + aT + 2.0 * T;
    const double A4 = A2 + 2.0 * T;
    const double mee[6] = {1.0, u2 + aT, ux2 + T, uy2 + T, ux2 * A4 + T * A2, uy2 * A4 + T * A2};
    const double moe[4] = {ux, ux * A2, ux * (ux2 + 3.0 * T), ux * (uy2 + T)};
    const double meo[4] = {uy, uy * A2, uy * (ux2 + T), uy * (uy2 + 3.0 * T)};
    const double moo[2] = {uxy, uxy * A4};
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        double s = K.iee[r][0];
#pragma unroll
        for (int c = 1; c < 6; ++c) s = fma(K.iee[r][c], mee[c], s);
        h.ee[r] = m.rho * s;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double so = 0.0, se = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            so = fma(K.ioe[r][c], moe[c], so);
            se = fma(K.ieo[r][c], meo[c], se);
        }
        h.oe[r] = m.rho * so;
        h.eo[r] = m.rho * se;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) h.oo[r] = m.rho * fma(K.ioo[r][0], moo[0], K.ioo[r][1] * moo[1]);
}

// Minmod selection of Eq. (16) as (alpha, beta) in {0, 1}.
template <typename R>
__device__ __forceinline__ void minmod_select(R X, R Y, double& alpha, double& beta) {
    const bool same = (X > R(0) && Y > R(0)) || (X < R(0) && Y < R(0));
    const bool first = fabs((double)X) <= fabs((double)Y);
    alpha = (same && first) ? 1.0 : 0.0;
    beta = (same && !first) ? 1.0 : 0.0;
}

struct Quad {
    double rho, ux, uy, T;
};

// (d f^eq / d q)^T a for q = (rho, u_x, u_y, T) at the state m, from the
// parity transform hb = P^T a of a: w = B^T hb and its products with the
// raw moments and their derivatives, one parity block at a time (ee, then oe
// and eo, then oo) with the scheduler kept from interleaving the blocks, so
// that only one block's weights and tables are live at once.
__device__ __forceinline__ Quad equilibrium_vjp_q_parity(const Macro& m, const KParams& K,
                                                        double a, const Parity& hb) {
    const double ux = m.ux, uy = m.uy, T = m.T;
    const double ux2 = ux * ux, uy2 = uy * uy, u2 = ux2 + uy2, uxy = ux * uy;
    const double A2 = u2 + (a + 2.0) * T, A4 = u2 + (a + 4.0) * T;
    double gr = 0.0, gx = 0.0, gy = 0.0, gT = 0.0;
    {
        double wee[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < 6; ++r) s = fma(K.iee[r][c], hb.ee[r], s);
            wee[c] = s;
        }
        const double mee[6] = {1.0, u2 + a * T, ux2 + T, uy2 + T, ux2 * A4 + T * A2,
                               uy2 * A4 + T * A2};
        const double ee_x[6] = {0.0, 2.0 * ux, 2.0 * ux, 0.0, 2.0 * ux * (A4 + ux2 + T),
                                2.0 * ux * (uy2 + T)};
        const double ee_y[6] = {0.0, 2.0 * uy, 0.0, 2.0 * uy, 2.0 * uy * (ux2 + T),
                                2.0 * uy * (A4 + uy2 + T)};
        const double ee_T[6] = {0.0, a, 1.0, 1.0, ux2 * (a + 4.0) + A2 + T * (a + 2.0),
                                uy2 * (a + 4.0) + A2 + T * (a + 2.0)};
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            gr = fma(wee[c], mee[c], gr);
            gx = fma(wee[c], ee_x[c], gx);
            gy = fma(wee[c], ee_y[c], gy);
            gT = fma(wee[c], ee_T[c], gT);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    {
        double woe[4], weo[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double so = 0.0, se = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                so = fma(K.ioe[r][c], hb.oe[r], so);
                se = fma(K.ieo[r][c], hb.eo[r], se);
            }
            woe[c] = so;
            weo[c] = se;
        }
        const double moe[4] = {ux, ux * A2, ux * (ux2 + 3.0 * T), ux * (uy2 + T)};
        const double meo[4] = {uy, uy * A2, uy * (ux2 + T), uy * (uy2 + 3.0 * T)};
        const double oe_x[4] = {1.0, A2 + 2.0 * ux2, 3.0 * (ux2 + T), uy2 + T};
        const double oe_y[4] = {0.0, 2.0 * uxy, 0.0, 2.0 * uxy};
        const double oe_T[4] = {0.0, ux * (a + 2.0), 3.0 * ux, ux};
        const double eo_x[4] = {0.0, 2.0 * uxy, 2.0 * uxy, 0.0};
        const double eo_y[4] = {1.0, A2 + 2.0 * uy2, ux2 + T, 3.0 * (uy2 + T)};
        const double eo_T[4] = {0.0, uy * (a + 2.0), uy, 3.0 * uy};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            gr = fma(woe[c], moe[c], fma(weo[c], meo[c], gr));
            gx = fma(woe[c], oe_x[c], fma(weo[c], eo_x[c], gx));
            gy = fma(woe[c], oe_y[c], fma(weo[c], eo_y[c], gy));
            gT = fma(woe[c], oe_T[c], fma(weo[c], eo_T[c], gT));
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    {
        double woo[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) woo[c] = fma(K.ioo[0][c], hb.oo[0], K.ioo[1][c] * hb.oo[1]);
        const double moo[2] = {uxy, uxy * A4};
        const double oo_x[2] = {uy, uy * (A4 + 2.0 * ux2)};
        const double oo_y[2] = {ux, ux * (A4 + 2.0 * uy2)};
        const double oo_T[2] = {0.0, uxy * (a + 4.0)};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            gr = fma(woo[c], moo[c], gr);
            gx = fma(woo[c], oo_x[c], gx);
            gy = fma(woo[c], oo_y[c], gy);
            gT = fma(woo[c], oo_T[c], gT);
        }
    }
    return Quad{gr, m.rho * gx, m.rho * gy, m.rho * gT};
}

// (d f^eq / d q)^T a for q = (rho, u_x, u_y, T) at the state m.
__device__ __forceinline__ Quad equilibrium_vjp_q(const Macro& m, const KParams& K, double a,
                                                 const double adj[NV]) {
    Parity hb;
    to_parity(adj, hb);   // P^T a
    return equilibrium_vjp_q_parity(m, K, a, hb);
}

// (d q / d f)^T g at the state m, velocity k: q = (rho, u_x, u_y, T).
__device__ __forceinline__ double moments_vjp_k(const Macro& m, const KParams& K, double a,
                                                const Quad& g, int k) {
    const double cx = K.vx[k] - m.ux, cy = K.vy[k] - m.uy;
    const double e = cx * cx + cy * cy + K.eta2[k];
    return g.rho + (g.ux * cx + g.uy * cy + g.T * (e - a * m.T) / a) / m.rho;
}

// The transposes read one velocity's state and adjoint along a line (x or y)
// through the cell, at offsets -3 .. 3 for the state and -2 .. 2 for the
// adjoint, held in registers.  Positions are offsets from the cell (local
// position 0); the global index of a position only decides which gathers a
// zero-gradient side skips.  Face selections: bit 0 alpha, bit 1 beta of
// minmod(F(l+1) - F(l), F(l) - F(l-1)) along the line (Eq. (16) branch
// order), at offsets -2 .. 2.  Offsets outside -2 .. 2 occur only in gathers
// that a zero-gradient side skips; they are clamped to keep every index in
// the arrays.
__device__ __forceinline__ constexpr int line_slot(int l) {
    return (l < -2 ? -2 : (l > 2 ? 2 : l)) + 2;
}
struct RegSel {
    unsigned char c[5];
    __device__ __forceinline__ void at(int l, double& al, double& be) const {
        const int k = c[line_slot(l)];
        al = (double)(k & 1);
        be = (double)(k >> 1);
    }
};
struct RegLine {
    double v[5];   // the adjoint, zero at zero-gradient ghosts
    __device__ __forceinline__ double at(int l) const { return v[line_slot(l)]; }
};

template <typename S>
__device__ __forceinline__ unsigned char face_code(S fm, S f0, S fp) {
    double al, be;
    minmod_select<S>(fp - f0, f0 - fm, al, be);
    return (unsigned char)((al != 0.0 ? 1 : 0) | (be != 0.0 ? 2 : 0));
}

// Gather of the NND transpose at local position lp, global position gp
// (see the header).
template <bool POS>
__device__ __forceinline__ double nnd_gather(const RegSel& Sl, const RegLine& A, int lp, int gp,
                                             int n, int bc) {
    double acc = 0.0;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int k = POS ? 1 - kk : 2 - kk;
        const int gx = gp - k;
        if (bc != CDBM_PERIODIC && (gx < 0 || gx >= n)) continue;
        const int l = lp - k;
        double coef;
        if (POS) {
            double a0, b0, a1, b1;   // s(l-1), s(l)
            Sl.at(l - 1, a0, b0);
            Sl.at(l, a1, b1);
            if (k == 1) coef = 0.5 * a1;
            else if (k == 0) coef = 1.0 + 0.5 * (b1 - a0 - a1);
            else if (k == -1) coef = -1.0 - 0.5 * (b1 - a0 + b0);
            else coef = 0.5 * b0;
        } else {
            double a1, b1, a2, b2;   // s(l), s(l+1)
            Sl.at(l, a1, b1);
            Sl.at(l + 1, a2, b2);
            if (k == 2) coef = -0.5 * a2;
            else if (k == 1) coef = 1.0 + 0.5 * (a2 - b2 + a1);
            else if (k == 0) coef = -1.0 + 0.5 * (b2 - a1 + b1);
            else coef = -0.5 * b1;
        }
        acc = fma(coef, A.at(l), acc);
    }
    return acc;
}

// Full NND transpose at the real cell of local position lc, global position
// gc, with the ghost aliases of a zero-gradient side folded in.
template <bool POS>
__device__ __forceinline__ double nnd_transpose(const RegSel& Sl, const RegLine& A, int lc, int gc,
                                                int n, int bc) {
    double acc = nnd_gather<POS>(Sl, A, lc, gc, n, bc);
    if (bc == CDBM_ZERO_GRADIENT) {
        if (gc == 0)
            acc += nnd_gather<POS>(Sl, A, lc - 1, -1, n, bc) +
                   nnd_gather<POS>(Sl, A, lc - 2, -2, n, bc);
        if (gc == n - 1)
            acc += nnd_gather<POS>(Sl, A, lc + 1, n, n, bc) +
                   nnd_gather<POS>(Sl, A, lc + 2, n + 1, n, bc);
    }
    return acc;
}

}  // namespace cdbm
