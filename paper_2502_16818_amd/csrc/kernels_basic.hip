// Point-wise and simple stencil kernels of the CDBM library: initial
// equilibrium, field checks, macroscopic moments, nonequilibrium measures,
// conserved totals and the unfused Runge-Kutta stage.
#include <hip/hip_runtime.h>

#include "cell.hpp"
#include "launch.hpp"
#include "step_fused.hpp"

namespace cdbm {

namespace {

// f = f^eq(rho, u, T) per cell (the initial condition of Sec. 3).
template <typename S>
__global__ void __launch_bounds__(256) k_init(const double* __restrict__ rho,
                                              const double* __restrict__ ux,
                                              const double* __restrict__ uy,
                                              const double* __restrict__ T, S* __restrict__ f,
                                              KParams K, int64_t cells) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    Macro m{rho[c], ux[c], uy[c], T[c]};
    double feq[NV];
    equilibrium(m, K, K.a, feq);
#pragma unroll
    for (int i = 0; i < NV; ++i) f[i * cells + c] = (S)feq[i];
}

// bad |= 1 if rho <= 0, T <= 0 or any field value is not finite.
__global__ void __launch_bounds__(256) k_check_fields(const double* __restrict__ rho,
                                                      const double* __restrict__ ux,
                                                      const double* __restrict__ uy,
                                                      const double* __restrict__ T,
                                                      int64_t cells, int* __restrict__ bad) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const double r = rho[c], a = ux[c], b = uy[c], t = T[c];
    const bool ok = isfinite(r) && isfinite(a) && isfinite(b) && isfinite(t) && r > 0.0 && t > 0.0;
    if (!ok) atomicOr(bad, 1);
}

template <typename S>
__device__ __forceinline__ void load_cell(const S* __restrict__ f, int64_t cells, int64_t c,
                                          double fd[NV]) {
#pragma unroll
    for (int i = 0; i < NV; ++i) fd[i] = (double)f[i * cells + c];
}

// The compensated mixed form (CDBM_MIXED_COMP): a state holds the 16 planes
// of f in float and then the four planes of r, the part of the cell's
// (rho, j_x, j_y, 2E) that float storage of f rounded off.

// (rho, j_x, j_y, 2E) of the distributions whose parity combinations are g.
__device__ __forceinline__ void conserved_of(const Parity& g, const KParams& K, double out[4]) {
    out[0] = ((g.ee[0] + g.ee[1]) + (g.ee[2] + g.ee[3])) + (g.ee[4] + g.ee[5]);
    double jx = 0.0, jy = 0.0, e2 = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        jx = fma(K.jx[c], g.oe[c], jx);
        jy = fma(K.jy[c], g.eo[c], jy);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) e2 = fma(K.en[c], g.ee[c], e2);
    out[1] = jx;
    out[2] = jy;
    out[3] = e2;
}

// Macroscopic fields of a compensated cell: the conserved moments of its
// stored f plus its residual r.
__device__ __forceinline__ Macro macro_compensated(const Parity& g, const double r[4],
                                                   const KParams& K) {
    double q[4];
    conserved_of(g, K, q);
    const double rho = q[0] + r[0];
    Macro m;
    m.rho = rho;
    m.ux = (q[1] + r[1]) / rho;
    m.uy = (q[2] + r[2]) / rho;
    m.T = ((q[3] + r[3]) / rho - (m.ux * m.ux + m.uy * m.uy)) * K.inv_a;
    return m;
}

__device__ __forceinline__ void load_residual(const float* __restrict__ f, int64_t cells,
                                              int64_t c, double r[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = (double)f[(NV + k) * cells + c];
}

// An empty asm statement that takes the values as register operands: every
// load feeding them completes before it, and none of them is used before
// it, so the loads are issued together rather than one at a time.
__device__ __forceinline__ void hold_values(float (&v)[4]) {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]));
}
__device__ __forceinline__ void hold_values(float (&v)[NV + 4]) {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]),
                 "+v"(v[6]), "+v"(v[7]), "+v"(v[8]), "+v"(v[9]));
    asm volatile("" : "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]), "+v"(v[14]),
                 "+v"(v[15]), "+v"(v[16]), "+v"(v[17]), "+v"(v[18]), "+v"(v[19]));
}
__device__ __forceinline__ void hold_values(float (&v)[4][6]) {
    asm volatile("" : "+v"(v[0][0]), "+v"(v[0][1]), "+v"(v[0][2]), "+v"(v[0][3]), "+v"(v[0][4]),
                 "+v"(v[0][5]), "+v"(v[1][0]), "+v"(v[1][1]), "+v"(v[1][2]), "+v"(v[1][3]),
                 "+v"(v[1][4]), "+v"(v[1][5]));
    asm volatile("" : "+v"(v[2][0]), "+v"(v[2][1]), "+v"(v[2][2]), "+v"(v[2][3]), "+v"(v[2][4]),
                 "+v"(v[2][5]), "+v"(v[3][0]), "+v"(v[3][1]), "+v"(v[3][2]), "+v"(v[3][3]),
                 "+v"(v[3][4]), "+v"(v[3][5]));
}

// Compensated initial state: f = f^eq rounded to float, r = the conserved
// moments of what the rounding removed.
__global__ void __launch_bounds__(256) k_init_comp(const double* __restrict__ rho,
                                                   const double* __restrict__ ux,
                                                   const double* __restrict__ uy,
                                                   const double* __restrict__ T,
                                                   float* __restrict__ f, KParams K,
                                                   int64_t cells) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    Macro m{rho[c], ux[c], uy[c], T[c]};
    double feq[NV], lost[NV];
    equilibrium(m, K, K.a, feq);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const float v = (float)feq[i];
        f[i * cells + c] = v;
        lost[i] = feq[i] - (double)v;
    }
    Parity g;
    to_parity(lost, g);
    double r[4];
    conserved_of(g, K, r);
#pragma unroll
    for (int k = 0; k < 4; ++k) f[(NV + k) * cells + c] = (float)r[k];
}

template <typename S, bool COMP = false>
__global__ void __launch_bounds__(256) k_moments(const S* __restrict__ f, double* __restrict__ rho,
                                                 double* __restrict__ ux, double* __restrict__ uy,
                                                 double* __restrict__ T, KParams K, int64_t cells) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    double fd[NV];
    load_cell(f, cells, c, fd);
    Parity g;
    to_parity(fd, g);
    Macro m;
    if constexpr (COMP) {
        double r[4];
        load_residual(f, cells, c, r);
        m = macro_compensated(g, r, K);
    } else {
        m = macro_from_parity(g, K, K.inv_a);
    }
    rho[c] = m.rho;
    ux[c] = m.ux;
    uy[c] = m.uy;
    T[c] = m.T;
}

// Eqs. (8)-(11): sum_i (f_i - f_i^eq) Psi_r(v_i - u), rows r = 5..16.
// RAW: the measures of the raw-moment construction, Psi_r(v_i) at the raw
// velocities (same f^eq).
// COMP: f^eq of the compensated moments, f the stored float distributions.
template <typename S, bool RAW, bool COMP = false>
__global__ void __launch_bounds__(256) k_tne(const S* __restrict__ f, double* __restrict__ out,
                                             KParams K, int64_t cells) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    double fd[NV];
    load_cell(f, cells, c, fd);
    Parity g;
    to_parity(fd, g);
    Macro m;
    if constexpr (COMP) {
        double r[4];
        load_residual(f, cells, c, r);
        m = macro_compensated(g, r, K);
    } else {
        m = macro_from_parity(g, K, K.inv_a);
    }
    double feq[NV];
    equilibrium(m, K, K.a, feq);
    double acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const double d = fd[i] - feq[i];
        const double cx = RAW ? K.vx[i] : K.vx[i] - m.ux, cy = RAW ? K.vy[i] : K.vy[i] - m.uy;
        const double e = cx * cx + cy * cy + K.eta2[i];
        const double xx = cx * cx, xy = cx * cy, yy = cy * cy;
        acc[0] = fma(d, xx, acc[0]);
        acc[1] = fma(d, xy, acc[1]);
        acc[2] = fma(d, yy, acc[2]);
        acc[3] = fma(d, e * cx, acc[3]);
        acc[4] = fma(d, e * cy, acc[4]);
        acc[5] = fma(d, xx * cx, acc[5]);
        acc[6] = fma(d, xx * cy, acc[6]);
        acc[7] = fma(d, xy * cy, acc[7]);
        acc[8] = fma(d, yy * cy, acc[8]);
        acc[9] = fma(d, e * xx, acc[9]);
        acc[10] = fma(d, e * xy, acc[10]);
        acc[11] = fma(d, e * yy, acc[11]);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k * cells + c] = acc[k];
}

// Per-block partial sums of (rho, j_x, j_y, 2E); block count is fixed.
template <typename S, bool COMP = false>
__global__ void __launch_bounds__(256) k_totals_partial(const S* __restrict__ f, KParams K,
                                                        int64_t cells, double* __restrict__ part) {
    __shared__ double red[4][256];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells;
         c += (int64_t)gridDim.x * blockDim.x) {
        double fd[NV];
        load_cell(f, cells, c, fd);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            acc[0] += fd[i];
            acc[1] = fma(fd[i], K.vx[i], acc[1]);
            acc[2] = fma(fd[i], K.vy[i], acc[2]);
            acc[3] = fma(fd[i], K.vx[i] * K.vx[i] + K.vy[i] * K.vy[i] + K.eta2[i], acc[3]);
        }
        if constexpr (COMP) {
            double r[4];
            load_residual(f, cells, c, r);
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] += r[k];
        }
    }
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// out[k] = sum over blocks of part[b*4 + k], in a fixed order.
__global__ void __launch_bounds__(256) k_sum_partials(const double* __restrict__ part, int nblocks,
                                                      int ncomp, double* __restrict__ out) {
    __shared__ double red[256];
    for (int k = 0; k < ncomp; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += part[b * ncomp + k];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = red[0];
        __syncthreads();
    }
}

// Global-memory neighbour access with boundary conditions, for the unfused stage.
template <typename S>
struct GlobalLd {
    const S* __restrict__ f;
    int64_t cells;
    int nx;
    int xs[5];   // source columns of offsets -2..2
    int ys[5];   // source rows of offsets -2..2
    __device__ __forceinline__ S operator()(int i, int ox, int oy) const {
        return f[i * cells + (int64_t)ys[oy + 2] * nx + xs[ox + 2]];
    }
};

// One Runge-Kutta stage without fusion, with the same per-cell arithmetic
// as the fused step:
//   STAGE2 == false:  out = f + dt L(f)
//   STAGE2 == true:   out = base / 2 + (f + dt L(f)) / 2
template <typename S, bool STAGE2>
__global__ void __launch_bounds__(256) k_stage(const S* __restrict__ fin, const S* __restrict__ base,
                                               S* __restrict__ fout,
                                               const KParams* __restrict__ Kd) {
    const KParams& K = *Kd;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= K.nx || y >= K.ny) return;
    const int64_t cells = (int64_t)K.nx * K.ny;
    GlobalLd<S> ld;
    ld.f = fin;
    ld.cells = cells;
    ld.nx = K.nx;
#pragma unroll
    for (int o = -2; o <= 2; ++o) {
        ld.xs[o + 2] = wrap_or_clamp(x + o, K.nx, K.bcx);
        ld.ys[o + 2] = wrap_or_clamp(y + o, K.ny, K.bcy);
    }
    S out[NV];
    stage_cell_k<S, STAGE2>(ld, K, out);
    const int64_t c = (int64_t)y * K.nx + x;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        S v = out[i];
        if (STAGE2) v = fma(S(0.5), base[i * cells + c], v);
        fout[i * cells + c] = v;
    }
}

// One Runge-Kutta stage of the compensated form, one cell per thread: f is
// read from float storage and every term is formed in double, as in the
// FP64 form:
//   STAGE2 == false:  y = f + A,              out = round(y + C),
//                     r_out = r + m(y - out)
//   STAGE2 == true:   y = base/2 + f/2 + A,   out = round(y + C),
//                     r_out = r_base/2 + r/2 + m(y - out)
// where A is the stage's advection term dt (-v . grad f) of Eqs. (12)-(20)
// and C its relaxation term -dt (f - f^eq)/tau of Eq. (1) (both halved in
// the second stage), f^eq is that of the compensated moments m(f) + r, and
// m(.) is (rho, j_x, j_y, 2E) of a set of 16 values.  The conserved moments
// m(f) + r of the output are those of the stage's combination without C
// (the advection flux changes them, the relaxation does not); C itself
// carries dt/tau of r into f.  The differences of the NND stencil are exact
// in double (two floats of like size), so the advection terms of
// neighbouring cells cancel in the grid sums to FP64 rounding.
template <bool STAGE2>
__global__ void __launch_bounds__(256) k_stage_comp(const float* __restrict__ fin,
                                                    const float* __restrict__ base,
                                                    float* __restrict__ fout,
                                                    const KParams* __restrict__ Kd) {
    const KParams& K = *Kd;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= K.nx || y >= K.ny) return;
    const int64_t cells = (int64_t)K.nx * K.ny;
    GlobalLd<float> ld;
    ld.f = fin;
    ld.cells = cells;
    ld.nx = K.nx;
#pragma unroll
    for (int o = -2; o <= 2; ++o) {
        ld.xs[o + 2] = wrap_or_clamp(x + o, K.nx, K.bcx);
        ld.ys[o + 2] = wrap_or_clamp(y + o, K.ny, K.bcy);
    }
    const int64_t c = (int64_t)y * K.nx + x;
    // The loads of a cell's 16 values and residual, and then of each group's
    // stencils, are issued together and held by one empty asm statement
    // before any is used: left to itself the compiler fetched one value at a
    // time (load, wait, convert) to save registers, and the stage took twice
    // as long.
    float f[NV + 4];
#pragma unroll
    for (int i = 0; i < NV; ++i) f[i] = ld(i, 0, 0);
#pragma unroll
    for (int k = 0; k < 4; ++k) f[NV + k] = fin[(NV + k) * cells + c];
    hold_values(f);
    double fd[NV], r[4];
#pragma unroll
    for (int i = 0; i < NV; ++i) fd[i] = (double)f[i];
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = (double)f[NV + k];
    Parity g;
    to_parity(fd, g);
    const Macro m = macro_compensated(g, r, K);
    double neq[NV];
    nonequilibrium(g, m, K, K.a, neq);
    const double nza = K.nzq[STAGE2][0], nzd = K.nzq[STAGE2][1];
    double lost[NV];
    // groups of four velocities (axis group: one stencil direction each,
    // diagonal group: two); st[k][0..2] the x stencil of velocity i0 + k
    // without its centre, st[k][3..5] the y stencil, upwind first
#pragma unroll
    for (int i0 = 0; i0 < NV; i0 += 4) {
        float st[4][6];
        float hb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = i0 + k;
            if (SX[i] > 0) {
                st[k][0] = ld(i, -2, 0); st[k][1] = ld(i, -1, 0); st[k][2] = ld(i, 1, 0);
            } else if (SX[i] < 0) {
                st[k][0] = ld(i, -1, 0); st[k][1] = ld(i, 1, 0); st[k][2] = ld(i, 2, 0);
            } else {
                st[k][0] = st[k][1] = st[k][2] = 0.0f;
            }
            if (SY[i] > 0) {
                st[k][3] = ld(i, 0, -2); st[k][4] = ld(i, 0, -1); st[k][5] = ld(i, 0, 1);
            } else if (SY[i] < 0) {
                st[k][3] = ld(i, 0, -1); st[k][4] = ld(i, 0, 1); st[k][5] = ld(i, 0, 2);
            } else {
                st[k][3] = st[k][4] = st[k][5] = 0.0f;
            }
            hb[k] = STAGE2 ? base[i * cells + c] : 0.0f;
        }
        hold_values(st);
        if (STAGE2) hold_values(hb);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = i0 + k;
            const double cx = STAGE2 ? K.cxh[i] : K.cx[i];
            const double cy = STAGE2 ? K.cyh[i] : K.cy[i];
            double adv = 0.0;
            if (SX[i] > 0)
                adv = cx * nnd_pos<double>(st[k][0], st[k][1], fd[i], st[k][2]);
            else if (SX[i] < 0)
                adv = cx * nnd_neg<double>(st[k][0], fd[i], st[k][1], st[k][2]);
            if (SY[i] > 0)
                adv += cy * nnd_pos<double>(st[k][3], st[k][4], fd[i], st[k][5]);
            else if (SY[i] < 0)
                adv += cy * nnd_neg<double>(st[k][3], fd[i], st[k][4], st[k][5]);
            const double coll = ((i & 4) ? nzd : nza) * neq[i];
            double yv = adv;
            if (STAGE2) yv += 0.5 * fd[i] + 0.5 * (double)hb[k];
            else yv += fd[i];
            const float o = (float)(yv + coll);
            fout[i * cells + c] = o;
            lost[i] = yv - (double)o;
        }
    }
    Parity gl;
    to_parity(lost, gl);
    double dm[4];
    conserved_of(gl, K, dm);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double rk = r[k];
        if (STAGE2) rk = 0.5 * (double)base[(NV + k) * cells + c] + 0.5 * rk;
        fout[(NV + k) * cells + c] = (float)(rk + dm[k]);
    }
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

template <typename S>
hipError_t launch_init(const double* rho, const double* ux, const double* uy, const double* T,
                       void* f, const KParams& K, hipStream_t st) {
    const int64_t cells = (int64_t)K.nx * K.ny;
    hipLaunchKernelGGL(k_init<S>, dim3(blocks_for(cells, 256)), dim3(256), 0, st, rho, ux, uy, T,
                       (S*)f, K, cells);
    return hipGetLastError();
}

hipError_t launch_check_fields(const double* rho, const double* ux, const double* uy,
                               const double* T, int64_t cells, int* bad, hipStream_t st) {
    hipLaunchKernelGGL(k_check_fields, dim3(blocks_for(cells, 256)), dim3(256), 0, st, rho, ux, uy,
                       T, cells, bad);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_moments(const void* f, double* rho, double* ux, double* uy, double* T,
                          const KParams& K, hipStream_t st) {
    const int64_t cells = (int64_t)K.nx * K.ny;
    hipLaunchKernelGGL(k_moments<S>, dim3(blocks_for(cells, 256)), dim3(256), 0, st,
                       (const S*)f, rho, ux, uy, T, K, cells);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_tne(const void* f, double* out12, bool raw, const KParams& K, hipStream_t st) {
    const int64_t cells = (int64_t)K.nx * K.ny;
    if (raw)
        hipLaunchKernelGGL((k_tne<S, true>), dim3(blocks_for(cells, 256)), dim3(256), 0, st,
                           (const S*)f, out12, K, cells);
    else
        hipLaunchKernelGGL((k_tne<S, false>), dim3(blocks_for(cells, 256)), dim3(256), 0, st,
                           (const S*)f, out12, K, cells);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_totals(const void* f, double* partials, int nblocks, double* out4,
                         const KParams& K, hipStream_t st) {
    const int64_t cells = (int64_t)K.nx * K.ny;
    hipLaunchKernelGGL(k_totals_partial<S>, dim3(nblocks), dim3(256), 0, st, (const S*)f, K,
                       cells, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partials, nblocks, 4, out4);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double* part, int nblocks, int ncomp, double* out,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, part, nblocks, ncomp, out);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_stage(const void* fin, const void* base, void* fout, bool stage2,
                        const KParams& K, const KParams* Kd, hipStream_t st) {
    const dim3 grid(blocks_for(K.nx, 64), blocks_for(K.ny, 4));
    if (stage2)
        hipLaunchKernelGGL((k_stage<S, true>), grid, dim3(256), 0, st, (const S*)fin,
                           (const S*)base, (S*)fout, Kd);
    else
        hipLaunchKernelGGL((k_stage<S, false>), grid, dim3(256), 0, st, (const S*)fin,
                           (const S*)base, (S*)fout, Kd);
    return hipGetLastError();
}

hipError_t launch_init_comp(const double* rho, const double* ux, const double* uy,
                            const double* T, void* f, const KParams& K, hipStream_t st) {
    const int64_t cells = (int64_t)K.nx * K.ny;
    hipLaunchKernelGGL(k_init_comp, dim3(blocks_for(cells, 256)), dim3(256), 0, st, rho, ux, uy,
                       T, (float*)f, K, cells);
    return hipGetLastError();
}

hipError_t launch_moments_comp(const void* f, double* rho, double* ux, double* uy, double* T,
                               const KParams& K, hipStream_t st) {
    const int64_t cells = (int64_t)K.nx * K.ny;
    hipLaunchKernelGGL((k_moments<float, true>), dim3(blocks_for(cells, 256)), dim3(256), 0, st,
                       (const float*)f, rho, ux, uy, T, K, cells);
    return hipGetLastError();
}

hipError_t launch_tne_comp(const void* f, double* out12, bool raw, const KParams& K,
                           hipStream_t st) {
    const int64_t cells = (int64_t)K.nx * K.ny;
    if (raw)
        hipLaunchKernelGGL((k_tne<float, true, true>), dim3(blocks_for(cells, 256)), dim3(256), 0,
                           st, (const float*)f, out12, K, cells);
    else
        hipLaunchKernelGGL((k_tne<float, false, true>), dim3(blocks_for(cells, 256)), dim3(256), 0,
                           st, (const float*)f, out12, K, cells);
    return hipGetLastError();
}

hipError_t launch_totals_comp(const void* f, double* partials, int nblocks, double* out4,
                              const KParams& K, hipStream_t st) {
    const int64_t cells = (int64_t)K.nx * K.ny;
    hipLaunchKernelGGL((k_totals_partial<float, true>), dim3(nblocks), dim3(256), 0, st,
                       (const float*)f, K, cells, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partials, nblocks, 4, out4);
    return hipGetLastError();
}

hipError_t launch_stage_comp(const void* fin, const void* base, void* fout, bool stage2,
                             const KParams& K, const KParams* Kd, hipStream_t st) {
    const dim3 grid(blocks_for(K.nx, 64), blocks_for(K.ny, 4));
    if (stage2)
        hipLaunchKernelGGL((k_stage_comp<true>), grid, dim3(256), 0, st, (const float*)fin,
                           (const float*)base, (float*)fout, Kd);
    else
        hipLaunchKernelGGL((k_stage_comp<false>), grid, dim3(256), 0, st, (const float*)fin,
                           (const float*)base, (float*)fout, Kd);
    return hipGetLastError();
}

#define CDBM_INSTANTIATE(S)                                                                     \
    template hipError_t launch_init<S>(const double*, const double*, const double*,            \
                                       const double*, void*, const KParams&, hipStream_t);     \
    template hipError_t launch_moments<S>(const void*, double*, double*, double*, double*,     \
                                          const KParams&, hipStream_t);                        \
    template hipError_t launch_tne<S>(const void*, double*, bool, const KParams&, hipStream_t);      \
    template hipError_t launch_totals<S>(const void*, double*, int, double*, const KParams&,   \
                                         hipStream_t);                                         \
    template hipError_t launch_stage<S>(const void*, const void*, void*, bool, const KParams&, \
                                        const KParams*, hipStream_t);
CDBM_INSTANTIATE(float)
CDBM_INSTANTIATE(double)
#undef CDBM_INSTANTIATE

}  // namespace cdbm
