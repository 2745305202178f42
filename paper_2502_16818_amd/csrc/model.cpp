// Per-run constants of the CDBM step: velocity table, moment matrix at
// u = 0 and the inverses of its parity blocks.  See model.hpp.
#include "model.hpp"

#include <cmath>
#include <cstdio>
#include <cstring>

namespace cdbm {

namespace {

// Psi_r of Eq. (4) in the row order of Eq. (6), at velocity (cx, cy) and eta.
void moment_functions(double cx, double cy, double eta, double out[NV]) {
    const double e = cx * cx + cy * cy + eta * eta;
    out[0] = 1.0;
    out[1] = cx;
    out[2] = cy;
    out[3] = e;
    out[4] = cx * cx;
    out[5] = cx * cy;
    out[6] = cy * cy;
    out[7] = e * cx;
    out[8] = e * cy;
    out[9] = cx * cx * cx;
    out[10] = cx * cx * cy;
    out[11] = cx * cy * cy;
    out[12] = cy * cy * cy;
    out[13] = e * cx * cx;
    out[14] = e * cx * cy;
    out[15] = e * cy * cy;
}

// Gauss-Jordan inversion with partial pivoting in long double.  Returns false
// when a pivot vanishes relative to the matrix scale.
bool invert(int n, const double* A, double* Ainv, double* cond1) {
    long double m[6][12];
    double norm_a = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += std::fabs(A[i * n + j]);
        if (s > norm_a) norm_a = s;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j)
            m[i][j] = j < n ? (long double)A[i * n + j] : (long double)(j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabsl(m[r][c]) > fabsl(m[piv][c])) piv = r;
        if (!(fabsl(m[piv][c]) > 1e-300L * (long double)norm_a) || norm_a == 0.0) return false;
        if (piv != c)
            for (int j = 0; j < 2 * n; ++j) {
                long double t = m[c][j];
                m[c][j] = m[piv][j];
                m[piv][j] = t;
            }
        const long double d = m[c][c];
        for (int j = 0; j < 2 * n; ++j) m[c][j] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const long double f = m[r][c];
            if (f == 0.0L) continue;
            for (int j = 0; j < 2 * n; ++j) m[r][j] -= f * m[c][j];
        }
    }
    double norm_i = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) {
            Ainv[i * n + j] = (double)m[i][n + j];
            s += std::fabs(Ainv[i * n + j]);
        }
        if (s > norm_i) norm_i = s;
    }
    *cond1 = norm_a * norm_i;
    return std::isfinite(*cond1);
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

double extra_dof(double gamma) { return 2.0 / (gamma - 1.0) - 2.0; }

int build_params(const cdbm_params& p, KParams& k, std::string& err) {
    std::memset(&k, 0, sizeof(k));
    char buf[256];
    if (p.nx < 1 || p.ny < 1 || p.nx > 65536 || p.ny > 65536 ||
        (int64_t)p.nx * (int64_t)p.ny > (int64_t(1) << 28)) {
        std::snprintf(buf, sizeof buf, "grid %d x %d out of range (1..65536 each, <= 2^28 cells)",
                      p.nx, p.ny);
        err = buf;
        return CDBM_EINVAL;
    }
    if (!finite_pos(p.dx) || !finite_pos(p.dy) || !finite_pos(p.dt) || !finite_pos(p.tau)) {
        err = "dx, dy, dt and tau must be finite and positive";
        return CDBM_EINVAL;
    }
    if (p.dt / p.tau > 2.0) {
        std::snprintf(buf, sizeof buf, "dt/tau = %g exceeds 2, outside the stable interval of "
                      "the two-stage scheme for relaxation", p.dt / p.tau);
        err = buf;
        return CDBM_EINVAL;
    }
    if (p.dof_given != 0 && p.dof_given != 1) {
        err = "dof_given must be 0 (gamma given) or 1 (extra_dof given)";
        return CDBM_EINVAL;
    }
    if (p.dof_given == 0 && !(std::isfinite(p.gamma) && p.gamma > 1.0 && p.gamma <= 2.0)) {
        err = "gamma must lie in (1, 2] (I = 2/(gamma-1) - 2 >= 0)";
        return CDBM_EINVAL;
    }
    if (p.dof_given == 1 && !(std::isfinite(p.extra_dof) && p.extra_dof >= 0.0)) {
        err = "extra_dof (I) must be finite and >= 0";
        return CDBM_EINVAL;
    }
    for (int g = 0; g < 4; ++g) {
        if (!finite_pos(p.v[g])) {
            err = "discrete speeds v_a..v_d must be finite and positive";
            return CDBM_EINVAL;
        }
        if (!(std::isfinite(p.eta[g]) && p.eta[g] >= 0.0)) {
            err = "eta_a..eta_d must be finite and >= 0";
            return CDBM_EINVAL;
        }
    }
    if ((p.bc_x != CDBM_PERIODIC && p.bc_x != CDBM_ZERO_GRADIENT) ||
        (p.bc_y != CDBM_PERIODIC && p.bc_y != CDBM_ZERO_GRADIENT)) {
        err = "bc_x and bc_y must be CDBM_PERIODIC or CDBM_ZERO_GRADIENT";
        return CDBM_EINVAL;
    }
    if (p.precision != CDBM_FP64 && p.precision != CDBM_MIXED && p.precision != CDBM_MIXED_COMP) {
        err = "precision must be CDBM_FP64, CDBM_MIXED or CDBM_MIXED_COMP";
        return CDBM_EINVAL;
    }
    if (p.step_form < CDBM_STEP_AUTO || p.step_form > CDBM_STEP_FUSED2) {
        err = "step_form must be CDBM_STEP_AUTO, CDBM_STEP_FUSED, CDBM_STEP_SPLIT or "
              "CDBM_STEP_FUSED2";
        return CDBM_EINVAL;
    }
    if (p.step_form == CDBM_STEP_FUSED2 && p.precision != CDBM_MIXED) {
        err = "CDBM_STEP_FUSED2 needs CDBM_MIXED: four rings of FP64 rows do not fit the LDS";
        return CDBM_EINVAL;
    }
    if (p.precision == CDBM_MIXED_COMP && p.step_form != CDBM_STEP_AUTO &&
        p.step_form != CDBM_STEP_SPLIT) {
        err = "CDBM_MIXED_COMP runs as two single-stage launches: step_form must be "
              "CDBM_STEP_AUTO or CDBM_STEP_SPLIT";
        return CDBM_EINVAL;
    }

    // Velocity table, Eqs. (2)-(3).
    double vx[NV], vy[NV], eta[NV];
    for (int i = 0; i < NV; ++i) {
        const int g = i / 4;
        vx[i] = p.v[g] * SX[i];
        vy[i] = p.v[g] * SY[i];
        eta[i] = p.eta[g];
    }
    // M0[r][i] = Psi_r(v_i, eta_i), Eq. (6) at u = 0.
    double M0[NV][NV];
    for (int i = 0; i < NV; ++i) {
        double col[NV];
        moment_functions(vx[i], vy[i], eta[i], col);
        for (int r = 0; r < NV; ++r) M0[r][i] = col[r];
    }

    // Parity blocks: rows and representative columns.
    static const int ree[6] = {0, 3, 4, 6, 13, 15}, cee[6] = {0, 1, 4, 8, 9, 12};
    static const int roe[4] = {1, 7, 9, 11}, coe[4] = {0, 4, 8, 12};
    static const int reo[4] = {2, 8, 10, 12}, ceo[4] = {1, 4, 9, 12};
    static const int roo[2] = {5, 14}, coo[2] = {4, 12};
    // Unpacking scale of each parity unknown: 1/2 for axis groups, 1/4 for diagonal ones.
    static const double see[6] = {0.5, 0.5, 0.25, 0.5, 0.5, 0.25};
    static const double soe[4] = {0.5, 0.25, 0.5, 0.25};
    static const double soo[2] = {0.25, 0.25};

    // Check that M0 really is block diagonal in this basis: every entry must
    // follow from its block entry by the sign pattern of the combination.
    for (int r = 0; r < NV; ++r) {
        const bool odd_x = (r == 1 || r == 7 || r == 9 || r == 11 || r == 5 || r == 14);
        const bool odd_y = (r == 2 || r == 8 || r == 10 || r == 12 || r == 5 || r == 14);
        for (int i = 0; i < NV; ++i) {
            const int g0 = (i / 4) * 4;
            const bool axis = ((i / 4) % 2) == 0;
            // representative column of velocity i for this row's parity
            int rep;
            if (axis)
                rep = (SX[i] != 0) ? g0 : g0 + 1;
            else
                rep = g0;
            double sign = 1.0;
            if (odd_x) sign *= (SX[i] < 0) ? -1.0 : 1.0;
            if (odd_y) sign *= (SY[i] < 0) ? -1.0 : 1.0;
            double expect = sign * M0[r][rep];
            if (axis && ((odd_x && SX[i] == 0) || (odd_y && SY[i] == 0))) expect = 0.0;
            if (M0[r][i] != expect) {
                err = "internal: moment matrix is not parity block diagonal";
                return CDBM_EINVAL;
            }
        }
    }

    auto block = [&](int n, const int* rows, const int* cols, const double* scale, double* inv,
                     const char* name) -> int {
        double B[36], Bi[36], cond = 0.0;
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) B[r * n + c] = M0[rows[r]][cols[c]];
        if (!invert(n, B, Bi, &cond) || cond > 1e10) {
            std::snprintf(buf, sizeof buf,
                          "moment matrix of the velocity set is singular or ill-conditioned "
                          "(%s parity block, 1-norm condition %.3g)", name, cond);
            err = buf;
            return CDBM_ESINGULAR;
        }
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) inv[r * n + c] = Bi[r * n + c] * scale[r];
        return CDBM_OK;
    };
    int rc;
    if ((rc = block(6, ree, cee, see, &k.iee[0][0], "even-even")) != CDBM_OK) return rc;
    if ((rc = block(4, roe, coe, soe, &k.ioe[0][0], "odd-even")) != CDBM_OK) return rc;
    if ((rc = block(4, reo, ceo, soe, &k.ieo[0][0], "even-odd")) != CDBM_OK) return rc;
    if ((rc = block(2, roo, coo, soo, &k.ioo[0][0], "odd-odd")) != CDBM_OK) return rc;

    // Mirror form of the even-even block (KParams::eep, ees); the x <-> y
    // symmetry it relies on holds for every velocity set of this model, so a
    // failure here is an internal error.
    {
        double scale = 0.0;
        for (int r = 0; r < 6; ++r)
            for (int c = 0; c < 6; ++c) scale = std::fmax(scale, std::fabs(k.iee[r][c]));
        static const int swap[6] = {0, 1, 3, 2, 5, 4};
        bool ok = true;
        for (int c = 0; c < 6; ++c) {
            ok = ok && std::fabs(k.iee[1][c] - k.iee[0][swap[c]]) <= 1e-12 * scale;
            ok = ok && std::fabs(k.iee[4][c] - k.iee[3][swap[c]]) <= 1e-12 * scale;
            ok = ok && std::fabs(k.iee[2][c] - k.iee[2][swap[c]]) <= 1e-12 * scale;
            ok = ok && std::fabs(k.iee[5][c] - k.iee[5][swap[c]]) <= 1e-12 * scale;
        }
        if (!ok) {
            err = "internal: even-even block is not symmetric under x <-> y";
            return CDBM_EINVAL;
        }
        for (int q = 0; q < 2; ++q) {
            const double* B = k.iee[3 * q];
            k.eep[q][0] = B[0];
            k.eep[q][1] = B[1];
            k.eep[q][2] = 0.5 * (B[2] + B[3]);
            k.eep[q][3] = 0.5 * (B[4] + B[5]);
            k.eep[q][4] = 0.5 * (B[2] - B[3]);
            k.eep[q][5] = 0.5 * (B[4] - B[5]);
            const double* D = k.iee[3 * q + 2];
            k.ees[q][0] = D[0];
            k.ees[q][1] = D[1];
            k.ees[q][2] = D[2];
            k.ees[q][3] = D[4];
        }
    }

    for (int c = 0; c < 4; ++c) {
        k.jx[c] = M0[1][coe[c]];
        k.jy[c] = M0[2][ceo[c]];
    }
    for (int c = 0; c < 6; ++c) k.en[c] = M0[3][cee[c]];
    for (int i = 0; i < NV; ++i) {
        k.vx[i] = vx[i];
        k.vy[i] = vy[i];
        k.eta2[i] = eta[i] * eta[i];
        k.cx[i] = -p.dt * vx[i] / p.dx;
        k.cy[i] = -p.dt * vy[i] / p.dy;
        k.cxf[i] = (float)k.cx[i];
        k.cyf[i] = (float)k.cy[i];
        k.cxh[i] = 0.5 * k.cx[i];
        k.cyh[i] = 0.5 * k.cy[i];
        k.cxhf[i] = (float)k.cxh[i];
        k.cyhf[i] = (float)k.cyh[i];
    }
    k.a = 2.0 + (p.dof_given ? p.extra_dof : extra_dof(p.gamma));
    k.inv_a = 1.0 / k.a;
    k.z = p.dt / p.tau;
    for (int h = 0; h < 2; ++h)
        for (int grp = 0; grp < 2; ++grp) {
            k.nzq[h][grp] = -k.z * (h ? 0.5 : 1.0) * (grp ? 0.25 : 0.5);
            k.nzqf[h][grp] = (float)k.nzq[h][grp];
        }
    k.dt = p.dt;
    k.tau = p.tau;
    k.nx = p.nx;
    k.ny = p.ny;
    k.bcx = p.bc_x;
    k.bcy = p.bc_y;
    return CDBM_OK;
}

}  // namespace cdbm
