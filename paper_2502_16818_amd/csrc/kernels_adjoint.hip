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
// A block handles ATX x ATY cells with AG groups of ATX x ATY threads.  The
// pointwise part (macroscopic state, equilibrium transpose, tau term) runs
// one thread per cell, split over two groups, and is shared through LDS.
// The NND transposes then run one velocity per group at a time (group k
// takes velocities k, k + AG, ...) on a tile of g_i and a_i with a 3-cell
// halo staged in LDS, so that every value a gather needs is loaded from HBM
// once per block instead of once per use, and the groups keep AG times as
// many waves busy as cells alone would.
template <typename S>
__global__ void __launch_bounds__(ATX * ATY * AG) k_stage_adjoint(const S* __restrict__ g,
                                                                  const double* __restrict__ a,
                                                                  const double* __restrict__ add,
                                                                  double* __restrict__ out,
                                                                  double w_in, double w_add,
                                                                  KParams K,
                                                                  double* __restrict__ tau_part) {
    constexpr int NC = ATX * ATY;               // cells per block
    constexpr int TILE = ATW * ATH;
    constexpr int PER = (TILE + NC - 1) / NC;   // tile elements per thread of a group
    __shared__ S Ft[AG][TILE];
    __shared__ double At[AG][TILE];
    __shared__ unsigned char Sx[AG][TILE], Sy[AG][TILE];   // face selections along x and y
    __shared__ double Mq[8][NC];                            // rho, u_x, u_y, T, then q
    __shared__ double red[NC];
    const int tid = threadIdx.x;
    const int grp = __builtin_amdgcn_readfirstlane(tid / NC);   // uniform per wave
    const int cid = tid % NC;
    const int lx = cid % ATX, ly = cid / ATX;
    const int x0 = blockIdx.x * ATX, y0 = blockIdx.y * ATY;
    const int x = x0 + lx, y = y0 + ly;
    const int nx = K.nx, ny = K.ny;
    const int64_t cells = (int64_t)nx * ny;
    const bool inside = x < nx && y < ny;

    // the tile elements this thread stages: source offset within a plane, or
    // a zero-gradient ghost (adjoint 0 there)
    int64_t src[PER];
    bool ghost[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int idx = cid + e * NC;
        const int tx = idx % ATW, ty = idx / ATW;
        const int gx = x0 - AH + tx, gy = y0 - AH + ty;
        src[e] = (int64_t)wrap_or_clamp(gy, ny, K.bcy) * nx + wrap_or_clamp(gx, nx, K.bcx);
        ghost[e] = (K.bcx != CDBM_PERIODIC && (gx < 0 || gx >= nx)) ||
                   (K.bcy != CDBM_PERIODIC && (gy < 0 || gy >= ny));
    }
    // tile values of the group's next velocity, loaded while the current one is used
    S fnext[PER];
    double anext[PER];
    auto fetch = [&](int i) {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            if (cid + e * NC < TILE) {
                fnext[e] = g[i * cells + src[e]];
                anext[e] = ghost[e] ? 0.0 : a[i * cells + src[e]];
            }
        }
    };
    // pointwise part: group 0 the state and the tau term, group 1 the
    // equilibrium transpose, both from the parity transforms pg = P g and
    // pa = P a (P P^T = k I per group, k = 2 axis, 4 diagonal).  With h the
    // parity form of f^eq (f^eq = P^T h), a . (g - f^eq) = pa . (pg / k - h).
    const int64_t c = (int64_t)y * nx + x;
    double tpart = 0.0;
    if (grp < 2 && inside) {
        Parity pg, pa;
        {
            double v[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) v[i] = (double)g[i * cells + c];
            to_parity(v, pg);
        }
        {
            double v[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) v[i] = a[i * cells + c];
            to_parity(v, pa);
        }
        const Macro m = macro_from_parity(pg, K, K.inv_a);
        if (grp == 0) {
            Parity h;
            equilibrium_parity(m, K, K.a, h);
            double d = 0.0;
#pragma unroll
            for (int r = 0; r < 6; ++r)
                d = fma(pa.ee[r], fma((r == 2 || r == 5) ? 0.25 : 0.5, pg.ee[r], -h.ee[r]), d);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double k = (r & 1) ? 0.25 : 0.5;
                d = fma(pa.oe[r], fma(k, pg.oe[r], -h.oe[r]), d);
                d = fma(pa.eo[r], fma(k, pg.eo[r], -h.eo[r]), d);
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) d = fma(pa.oo[r], fma(0.25, pg.oo[r], -h.oo[r]), d);
            tpart = (K.dt / (K.tau * K.tau)) * d;
            Mq[0][cid] = m.rho;
            Mq[1][cid] = m.ux;
            Mq[2][cid] = m.uy;
            Mq[3][cid] = m.T;
        } else {
            const Quad q = equilibrium_vjp_q_parity(m, K, K.a, pa);
            Mq[4][cid] = q.rho;
            Mq[5][cid] = q.ux;
            Mq[6][cid] = q.uy;
            Mq[7][cid] = q.T;
        }
    }
    fetch(grp);
    __syncthreads();
    Macro m{};
    Quad q{};
    if (inside) {
        m = Macro{Mq[0][cid], Mq[1][cid], Mq[2][cid], Mq[3][cid]};
        q = Quad{Mq[4][cid], Mq[5][cid], Mq[6][cid], Mq[7][cid]};
    }
    S* const F = Ft[grp];
    double* const Ag = At[grp];
    unsigned char* const Sxg = Sx[grp];
    unsigned char* const Syg = Sy[grp];
    const SelLine Srow{Sxg + (ly + AH) * ATW, 1}, Scol{Syg + lx + AH, ATW};
    const TileLine<double> Arow{Ag + (ly + AH) * ATW, 1}, Acol{Ag + lx + AH, ATW};
    // every group runs NV / AG iterations, so all threads meet every barrier
#pragma unroll 1
    for (int i = grp; i < NV; i += AG) {
        __syncthreads();   // the previous velocity's tiles are no longer read
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = cid + e * NC;
            if (idx < TILE) {
                F[idx] = fnext[e];
                Ag[idx] = anext[e];
            }
        }
        if (i + AG < NV) fetch(i + AG);
        __syncthreads();
        const int sx = SX[i & (NV - 1)], sy = SY[i & (NV - 1)];
        // selection of every tile position with both line neighbours in the tile
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = cid + e * NC;
            if (idx < TILE) {
                const int tx = idx % ATW, ty = idx / ATW;
                if (sx != 0 && tx > 0 && tx < ATW - 1)
                    Sxg[idx] = face_code<S>(F[idx - 1], F[idx], F[idx + 1]);
                if (sy != 0 && ty > 0 && ty < ATH - 1)
                    Syg[idx] = face_code<S>(F[idx - ATW], F[idx], F[idx + ATW]);
            }
        }
        __syncthreads();
        if (inside) {
            const double ceq = moments_vjp_k(m, K, K.a, q, i);
            double adv = 0.0;
            if (sx > 0)
                adv += K.cx[i] * nnd_transpose<true>(Srow, Arow, lx + AH, x, nx, K.bcx);
            else if (sx < 0)
                adv += K.cx[i] * nnd_transpose<false>(Srow, Arow, lx + AH, x, nx, K.bcx);
            if (sy > 0)
                adv += K.cy[i] * nnd_transpose<true>(Scol, Acol, ly + AH, y, ny, K.bcy);
            else if (sy < 0)
                adv += K.cy[i] * nnd_transpose<false>(Scol, Acol, ly + AH, y, ny, K.bcy);
            const double ai = Arow.at(lx + AH);   // a_i at the cell
            double v = ai + adv - K.z * (ai - ceq);
            v *= w_in;
            if (w_add != 0.0) v = fma(w_add, add[i * cells + c], v);
            out[i * cells + c] = v;
        }
    }
    if (grp == 0) red[cid] = tpart * w_in;
    __syncthreads();
    for (int s = NC / 2; s > 0; s >>= 1) {
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
    int b = threadIdx.x;
    // each thread's values in the order b, b + 256, ...; four loads in
    // flight at a time instead of one
    for (; b + 3 * 256 < n; b += 4 * 256) {
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = part[b + k * 256];
#pragma unroll
        for (int k = 0; k < 4; ++k) s += v[k];
    }
    for (; b < n; b += 256) s += part[b];
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
    hipLaunchKernelGGL(k_stage_adjoint<S>, grid, dim3(ATX * ATY * AG), 0, st, (const S*)g, (const double*)a,
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
