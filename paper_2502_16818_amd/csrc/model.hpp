// Host-side construction of the per-run constants of the CDBM step.
//
// The equilibrium of Eq. (7) is f^eq = M(u)^{-1} fbar^eq with M(u) the
// 16x16 matrix of Eq. (6) evaluated at the peculiar velocities v_i - u.
// Every row Psi_r(v - u) expands into rows of the same list with degree <= r
// (a binomial shift), so M(u) = S(u) M0 with S(u) unit lower triangular and
// M0 = M(0); then f^eq = M0^{-1} m^eq where m^eq = S(u)^{-1} fbar^eq is the
// vector of raw Maxwellian moments.  M0 depends only on the velocity set,
// so it is inverted once per run, here, and every cell applies the same
// inverse.
//
// The velocity set is symmetric under x -> -x and y -> -y.  In the basis of
// parity combinations of each group of four distributions, M0 is exactly
// block diagonal: a 6x6 block of rows even in both components
// (1, 4, 5, 7, 14, 16), two 4x4 blocks odd in one component
// (2, 8, 10, 12 and 3, 9, 11, 13) and a 2x2 block odd in both (6, 15).
// Those blocks are what the kernels contract with (72 multiply-adds per cell
// instead of 256).
#pragma once

#include <cstdint>
#include <string>

#include "../../include/cdbm.h"

namespace cdbm {

constexpr int NV = 16;

// Direction signs of the 16 discrete velocities (Eq. (2), axis groups a and
// c read as v(1,0), v(0,1), v(-1,0), v(0,-1); diagonal groups b and d as
// v(1,1), v(-1,1), v(-1,-1), v(1,-1)).
constexpr int SX[NV] = {1, 0, -1, 0, 1, -1, -1, 1, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int SY[NV] = {0, 1, 0, -1, 1, 1, -1, -1, 0, 1, 0, -1, 1, 1, -1, -1};

// Constants handed by value to every kernel.
struct KParams {
    // Inverses of the parity blocks of M0.  Output rows are pre-multiplied by
    // 1/2 (axis groups) or 1/4 (diagonal groups), so that the unpacking of
    // parity combinations into the 16 distributions is additions only.
    double iee[6][6];
    double ioe[4][4];
    double ieo[4][4];
    double ioo[2][2];
    // The even-even block in mirror form.  The velocity set is symmetric under
    // x <-> y, which swaps unknowns 0 <-> 1 and 3 <-> 4 of the block (the
    // axis pairs of groups a and c), keeps 2 and 5 (the diagonal groups), and
    // swaps moments 2 <-> 3 and 4 <-> 5; so row 1 of iee is row 0 with those
    // columns swapped, row 4 likewise row 3, and rows 2 and 5 weigh each
    // swapped pair equally.  eep[p] (pairs p = 0: rows 0, 1; p = 1: rows 3, 4)
    // holds {B0, B1, (B2 + B3) / 2, (B4 + B5) / 2, (B2 - B3) / 2, (B4 - B5) / 2}
    // of the pair's first row B, and ees[p] (rows 2, 5) {B0, B1, B2, B4}.
    double eep[2][6];
    double ees[2][4];
    // Rows of M0 in the parity basis that give the conserved moments:
    // j_x = sum jx[k] g_oe[k], j_y = sum jy[k] g_eo[k], 2E = sum en[k] g_ee[k]
    // (rho = sum of the six even-even combinations).
    double jx[4], jy[4], en[6];
    double vx[NV], vy[NV], eta2[NV];
    double cx[NV], cy[NV];     // -dt v_ix / dx and -dt v_iy / dy
    float cxf[NV], cyf[NV];
    double cxh[NV], cyh[NV];   // the same halved (the second Runge-Kutta stage)
    float cxhf[NV], cyhf[NV];
    double a;                  // D + I
    double inv_a;              // 1 / (D + I)
    double z;                  // dt / tau
    // -z/2 (axis groups) and -z/4 (diagonal groups) for the first Runge-Kutta
    // stage, then halved for the second: the factors that turn the output of
    // nonequilibrium() into -z (f - f^eq).
    double nzq[2][2];
    float nzqf[2][2];
    double dt, tau;
    int32_t nx, ny, bcx, bcy;
};

// Validate p and fill k.  Returns CDBM_OK or an error code with a message.
int build_params(const cdbm_params& p, KParams& k, std::string& err);

// Field values the parameters define but the kernels do not need.
double extra_dof(double gamma);

}  // namespace cdbm
