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

// (d f^eq / d q)^T a for q = (rho, u_x, u_y, T) at the state m.
__device__ __forceinline__ Quad equilibrium_vjp_q(const Macro& m, const KParams& K, double a,
                                                 const double adj[NV]) {
    Parity hb;
    to_parity(adj, hb);   // P^T a
    // w = B^T hb per block
    double wee[6], woe[4], weo[4], woo[2];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < 6; ++r) s = fma(K.iee[r][c], hb.ee[r], s);
        wee[c] = s;
    }
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
#pragma unroll
    for (int c = 0; c < 2; ++c) woo[c] = fma(K.ioo[0][c], hb.oo[0], K.ioo[1][c] * hb.oo[1]);

    const double ux = m.ux, uy = m.uy, T = m.T;
    const double ux2 = ux * ux, uy2 = uy * uy, u2 = ux2 + uy2, uxy = ux * uy;
    const double A2 = u2 + (a + 2.0) * T, A4 = u2 + (a + 4.0) * T;
    // raw moments / rho and their derivatives, blocks (1,4,5,7,14,16),
    // (2,8,10,12), (3,9,11,13), (6,15)
    const double mee[6] = {1.0, u2 + a * T, ux2 + T, uy2 + T, ux2 * A4 + T * A2, uy2 * A4 + T * A2};
    const double moe[4] = {ux, ux * A2, ux * (ux2 + 3.0 * T), ux * (uy2 + T)};
    const double meo[4] = {uy, uy * A2, uy * (ux2 + T), uy * (uy2 + 3.0 * T)};
    const double moo[2] = {uxy, uxy * A4};
    const double ee_x[6] = {0.0, 2.0 * ux, 2.0 * ux, 0.0, 2.0 * ux * (A4 + ux2 + T),
                            2.0 * ux * (uy2 + T)};
    const double ee_y[6] = {0.0, 2.0 * uy, 0.0, 2.0 * uy, 2.0 * uy * (ux2 + T),
                            2.0 * uy * (A4 + uy2 + T)};
    const double ee_T[6] = {0.0, a, 1.0, 1.0, ux2 * (a + 4.0) + A2 + T * (a + 2.0),
                            uy2 * (a + 4.0) + A2 + T * (a + 2.0)};
    const double oe_x[4] = {1.0, A2 + 2.0 * ux2, 3.0 * (ux2 + T), uy2 + T};
    const double oe_y[4] = {0.0, 2.0 * uxy, 0.0, 2.0 * uxy};
    const double oe_T[4] = {0.0, ux * (a + 2.0), 3.0 * ux, ux};
    const double eo_x[4] = {0.0, 2.0 * uxy, 2.0 * uxy, 0.0};
    const double eo_y[4] = {1.0, A2 + 2.0 * uy2, ux2 + T, 3.0 * (uy2 + T)};
    const double eo_T[4] = {0.0, uy * (a + 2.0), uy, 3.0 * uy};
    const double oo_x[2] = {uy, uy * (A4 + 2.0 * ux2)};
    const double oo_y[2] = {ux, ux * (A4 + 2.0 * uy2)};
    const double oo_T[2] = {0.0, uxy * (a + 4.0)};
    double gr = 0.0, gx = 0.0, gy = 0.0, gT = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        gr = fma(wee[c], mee[c], gr);
        gx = fma(wee[c], ee_x[c], gx);
        gy = fma(wee[c], ee_y[c], gy);
        gT = fma(wee[c], ee_T[c], gT);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        gr = fma(woe[c], moe[c], fma(weo[c], meo[c], gr));
        gx = fma(woe[c], oe_x[c], fma(weo[c], eo_x[c], gx));
        gy = fma(woe[c], oe_y[c], fma(weo[c], eo_y[c], gy));
        gT = fma(woe[c], oe_T[c], fma(weo[c], eo_T[c], gT));
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        gr = fma(woo[c], moo[c], gr);
        gx = fma(woo[c], oo_x[c], gx);
        gy = fma(woo[c], oo_y[c], gy);
        gT = fma(woo[c], oo_T[c], gT);
    }
    return Quad{gr, m.rho * gx, m.rho * gy, m.rho * gT};
}

// (d q / d f)^T g at the state m, velocity k: q = (rho, u_x, u_y, T).
__device__ __forceinline__ double moments_vjp_k(const Macro& m, const KParams& K, double a,
                                                const Quad& g, int k) {
    const double cx = K.vx[k] - m.ux, cy = K.vy[k] - m.uy;
    const double e = cx * cx + cy * cy + K.eta2[k];
    return g.rho + (g.ux * cx + g.uy * cy + g.T * (e - a * m.T) / a) / m.rho;
}

// Accessor of one distribution along one axis of one grid, with the
// boundary map of the grid applied to extended positions.
template <typename S>
struct Line {
    const S* __restrict__ base;   // f_i (or a_i) at row/column 0 of the line
    int stride;                   // element stride between neighbours on the axis
    int n;                        // cells on the axis
    int bc;
    __device__ __forceinline__ int map(int p) const { return wrap_or_clamp(p, n, bc); }
    __device__ __forceinline__ S at(int p) const { return base[(int64_t)map(p) * stride]; }
};

// Face selection at cell x of the distribution on line F.
template <typename S>
__device__ __forceinline__ void face_sel(const Line<S>& F, int x, double& al, double& be) {
    const S fm = F.at(x - 1), f0 = F.at(x), fp = F.at(x + 1);
    minmod_select<S>(fp - f0, f0 - fm, al, be);
}

// Gather of the NND transpose at extended position p (see the header).
// F: the state (selections are taken in its own precision); A: the adjoint.
template <typename S, bool POS>
__device__ __forceinline__ double nnd_gather(const Line<S>& F, const Line<double>& A, int p) {
    double acc = 0.0;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int k = POS ? 1 - kk : 2 - kk;   // POS: +1, 0, -1, -2; else +2, +1, 0, -1
        int x = p - k;
        if (F.bc == CDBM_PERIODIC) {
            x = F.map(x);
        } else if (x < 0 || x >= F.n) {
            continue;
        }
        double coef;
        if (POS) {
            double a0, b0, a1, b1;   // s(x-1), s(x)
            face_sel(F, x - 1, a0, b0);
            face_sel(F, x, a1, b1);
            if (k == 1) coef = 0.5 * a1;
            else if (k == 0) coef = 1.0 + 0.5 * (b1 - a0 - a1);
            else if (k == -1) coef = -1.0 - 0.5 * (b1 - a0 + b0);
            else coef = 0.5 * b0;
        } else {
            double a1, b1, a2, b2;   // s(x), s(x+1)
            face_sel(F, x, a1, b1);
            face_sel(F, x + 1, a2, b2);
            if (k == 2) coef = -0.5 * a2;
            else if (k == 1) coef = 1.0 + 0.5 * (a2 - b2 + a1);
            else if (k == 0) coef = -1.0 + 0.5 * (b2 - a1 + b1);
            else coef = -0.5 * b1;
        }
        acc = fma(coef, A.at(x), acc);
    }
    return acc;
}

// Full NND transpose at real cell y (ghost aliases folded in).
template <typename S, bool POS>
__device__ __forceinline__ double nnd_transpose(const Line<S>& F, const Line<double>& A, int y) {
    double acc = nnd_gather<S, POS>(F, A, y);
    if (F.bc == CDBM_ZERO_GRADIENT) {
        if (y == 0) acc += nnd_gather<S, POS>(F, A, -1) + nnd_gather<S, POS>(F, A, -2);
        if (y == F.n - 1)
            acc += nnd_gather<S, POS>(F, A, F.n) + nnd_gather<S, POS>(F, A, F.n + 1);
    }
    return acc;
}

}  // namespace cdbm
