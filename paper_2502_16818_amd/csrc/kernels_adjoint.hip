// Reverse-mode kernels: transpose of one Runge-Kutta stage, of the initial
// equilibrium and of the macroscopic moments (see adjoint.hpp).
#include <hip/hip_runtime.h>

#include "adjoint.hpp"
#include "launch.hpp"

namespace cdbm {

namespace {

// out = w_add * add + w_in * E'(g)^T a, and the per-block partial sums of
// w_in * sum_i a_i dE_i/dtau = w_in * sum_i a_i dt (g_i - g_i^eq) / tau^2.
// The state g is in the storage precision S; adjoint vectors are double.
// A block handles ATX x ATY cells.  The pointwise part (equilibrium and
// moment transposes) reads the cell's 16 values directly; the NND transposes
// run one velocity at a time on a tile of g_i and a_i with a 3-cell halo
// staged in LDS, so that every value a gather needs is loaded from HBM once
// per block instead of once per use.
template <typename S>
__global__ void __launch_bounds__(ATX * ATY) k_stage_adjoint(const S* __restrict__ g,
                                                             const double* __restrict__ a,
                                                             const double* __restrict__ add,
                                                             double* __restrict__ out, double w_in,
                                                             double w_add, KParams K,
                                                             double* __restrict__ tau_part) {
    constexpr int NT = ATX * ATY;
    constexpr int TILE = ATW * ATH;
    constexpr int PER = (TILE + NT - 1) / NT;   // tile elements per thread
    __shared__ S Ft[TILE];
    __shared__ double At[TILE];
    __shared__ unsigned char Sx[TILE], Sy[TILE];   // face selections along x and y
    __shared__ double red[NT];
    const int tid = threadIdx.x;
    const int lx = tid % ATX, ly = tid / ATX;
    const int x0 = blockIdx.x * ATX, y0 = blockIdx.y * ATY;
    const int x = x0 + lx, y = y0 + ly;
    const int nx = K.nx, ny = K.ny;
    const int64_t cells = (int64_t)nx * ny;
    const bool inside = x < nx && y < ny;

    // the tile elements this thread stages: source offset within a plane, or
    // -1 for a zero-gradient ghost (adjoint 0 there)
    int64_t src[PER];
    bool ghost[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int idx = tid + e * NT;
        const int tx = idx % ATW, ty = idx / ATW;
        const int gx = x0 - AH + tx, gy = y0 - AH + ty;
        src[e] = (int64_t)wrap_or_clamp(gy, ny, K.bcy) * nx + wrap_or_clamp(gx, nx, K.bcx);
        ghost[e] = (K.bcx != CDBM_PERIODIC && (gx < 0 || gx >= nx)) ||
                   (K.bcy != CDBM_PERIODIC && (gy < 0 || gy >= ny));
    }

    // pointwise part: macroscopic state, equilibrium transpose and the tau term
    Macro m{};
    Quad q{};
    double tpart = 0.0;
    const int64_t c = (int64_t)y * nx + x;
    if (inside) {
        double gd[NV], ad[NV], feq[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            gd[i] = (double)g[i * cells + c];
            ad[i] = a[i * cells + c];
        }
        Parity pg;
        to_parity(gd, pg);
        m = macro_from_parity(pg, K, K.inv_a);
        equilibrium(m, K, K.a, feq);
        q = equilibrium_vjp_q(m, K, K.a, ad);
        const double tau2 = K.dt / (K.tau * K.tau);
#pragma unroll
        for (int i = 0; i < NV; ++i) tpart = fma(ad[i], tau2 * (gd[i] - feq[i]), tpart);
    }
    const SelLine Srow{Sx + (ly + AH) * ATW, 1}, Scol{Sy + lx + AH, ATW};
    const TileLine<double> Arow{At + (ly + AH) * ATW, 1}, Acol{At + lx + AH, ATW};
    // tile values of the next velocity, loaded while the current one is used
    S fnext[PER];
    double anext[PER];
    auto fetch = [&](int i) {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            if (tid + e * NT < TILE) {
                fnext[e] = g[i * cells + src[e]];
                anext[e] = ghost[e] ? 0.0 : a[i * cells + src[e]];
            }
        }
    };
    fetch(0);
    for (int i = 0; i < NV; ++i) {
        __syncthreads();   // the previous velocity's tiles are no longer read
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * NT;
            if (idx < TILE) {
                Ft[idx] = fnext[e];
                At[idx] = anext[e];
            }
        }
        if (i + 1 < NV) fetch(i + 1);
        __syncthreads();
        // selection of every tile position with both line neighbours in the tile
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * NT;
            if (idx < TILE) {
                const int tx = idx % ATW, ty = idx / ATW;
                if (SX[i] != 0 && tx > 0 && tx < ATW - 1)
                    Sx[idx] = face_code<S>(Ft[idx - 1], Ft[idx], Ft[idx + 1]);
                if (SY[i] != 0 && ty > 0 && ty < ATH - 1)
                    Sy[idx] = face_code<S>(Ft[idx - ATW], Ft[idx], Ft[idx + ATW]);
            }
        }
        __syncthreads();
        if (inside) {
            const double ceq = moments_vjp_k(m, K, K.a, q, i);
            double adv = 0.0;
            if (SX[i] != 0)
                adv += K.cx[i] * (SX[i] > 0 ? nnd_transpose<true>(Srow, Arow, lx + AH, x, nx, K.bcx)
                                            : nnd_transpose<false>(Srow, Arow, lx + AH, x, nx, K.bcx));
            if (SY[i] != 0)
                adv += K.cy[i] * (SY[i] > 0 ? nnd_transpose<true>(Scol, Acol, ly + AH, y, ny, K.bcy)
                                            : nnd_transpose<false>(Scol, Acol, ly + AH, y, ny, K.bcy));
            const double ai = Arow.at(lx + AH);   // a_i at the cell
            double v = ai + adv - K.z * (ai - ceq);
            v *= w_in;
            if (w_add != 0.0) v = fma(w_add, add[i * cells + c], v);
            out[i * cells + c] = v;
        }
    }
    tpart *= w_in;
    red[tid] = tpart;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) tau_part[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// dst[0] += scale * sum_b part[b], summed in a fixed order by one block.
__global__ void __launch_bounds__(256) k_accumulate(const double* __restrict__ part, int n,
                                                    double scale, double* __restrict__ dst) {
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < n; b += blockDim.x) s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) dst[0] += scale * red[0];
}

// g_q = (d f^eq(q) / d q)^T lam per cell.
template <typename S>
__global__ void __launch_bounds__(256) k_init_adjoint(const double* __restrict__ rho,
                                                      const double* __restrict__ ux,
                                                      const double* __restrict__ uy,
                                                      const double* __restrict__ T,
                                                      const double* __restrict__ lam,
                                                      double* __restrict__ g_rho,
                                                      double* __restrict__ g_ux,
                                                      double* __restrict__ g_uy,
                                                      double* __restrict__ g_T, KParams K,
                                                      int64_t cells) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    double ad[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) ad[i] = lam[i * cells + c];
    const Macro m{rho[c], ux[c], uy[c], T[c]};
    const Quad q = equilibrium_vjp_q(m, K, K.a, ad);
    g_rho[c] = q.rho;
    g_ux[c] = q.ux;
    g_uy[c] = q.uy;
    g_T[c] = q.T;
}

// lam_f = (d (rho, u, T) / d f)^T g per cell.
template <typename S>
__global__ void __launch_bounds__(256) k_moments_adjoint(const S* __restrict__ f,
                                                         const double* __restrict__ g_rho,
                                                         const double* __restrict__ g_ux,
                                                         const double* __restrict__ g_uy,
                                                         const double* __restrict__ g_T,
                                                         double* __restrict__ lam, KParams K,
                                                         int64_t cells) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    double fd[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) fd[i] = (double)f[i * cells + c];
    Parity pg;
    to_parity(fd, pg);
    const Macro m = macro_from_parity(pg, K, K.inv_a);
    const Quad q{g_rho[c], g_ux[c], g_uy[c], g_T[c]};
#pragma unroll
    for (int i = 0; i < NV; ++i) lam[i * cells + c] = moments_vjp_k(m, K, K.a, q, i);
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

int stage_adjoint_blocks(const KParams& K) {
    return (int)(blocks_for(K.nx, ATX) * blocks_for(K.ny, ATY));
}

template <typename S>
hipError_t launch_stage_adjoint(const void* g, const void* a, const void* add, void* out,
                                double* tau_part, double w_in, double w_add, const KParams& K,
                                hipStream_t st) {
    const dim3 grid(blocks_for(K.nx, ATX), blocks_for(K.ny, ATY));
    hipLaunchKernelGGL(k_stage_adjoint<S>, grid, dim3(ATX * ATY), 0, st, (const S*)g, (const double*)a,
                       (const double*)add, (double*)out, w_in, w_add, K, tau_part);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_init_adjoint(const double* rho, const double* ux, const double* uy,
                               const double* T, const void* lam, double* g_rho, double* g_ux,
                               double* g_uy, double* g_T, const KParams& K, hipStream_t st) {
    const int64_t cells = (int64_t)K.nx * K.ny;
    hipLaunchKernelGGL(k_init_adjoint<S>, dim3(blocks_for(cells, 256)), dim3(256), 0, st, rho, ux,
                       uy, T, (const double*)lam, g_rho, g_ux, g_uy, g_T, K, cells);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_moments_adjoint(const void* f, const double* g_rho, const double* g_ux,
                                  const double* g_uy, const double* g_T, void* lam,
                                  const KParams& K, hipStream_t st) {
    const int64_t cells = (int64_t)K.nx * K.ny;
    hipLaunchKernelGGL(k_moments_adjoint<S>, dim3(blocks_for(cells, 256)), dim3(256), 0, st,
                       (const S*)f, g_rho, g_ux, g_uy, g_T, (double*)lam, K, cells);
    return hipGetLastError();
}

hipError_t launch_accumulate_scalar(const double* part, int nblocks, double scale, double* dst,
                                    hipStream_t st) {
    hipLaunchKernelGGL(k_accumulate, dim3(1), dim3(256), 0, st, part, nblocks, scale, dst);
    return hipGetLastError();
}

#define CDBM_INSTANTIATE(S)                                                                      \
    template hipError_t launch_stage_adjoint<S>(const void*, const void*, const void*, void*,   \
                                                double*, double, double, const KParams&,        \
                                                hipStream_t);                                   \
    template hipError_t launch_init_adjoint<S>(const double*, const double*, const double*,     \
                                               const double*, const void*, double*, double*,    \
                                               double*, double*, const KParams&, hipStream_t);  \
    template hipError_t launch_moments_adjoint<S>(const void*, const double*, const double*,    \
                                                  const double*, const double*, void*,          \
                                                  const KParams&, hipStream_t);
CDBM_INSTANTIATE(float)
CDBM_INSTANTIATE(double)
#undef CDBM_INSTANTIATE

}  // namespace cdbm
