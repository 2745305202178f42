// Reverse-mode kernels: transpose of one Runge-Kutta stage, of the initial
// equilibrium and of the macroscopic moments (see adjoint.hpp).
#include <hip/hip_runtime.h>

#include "adjoint.hpp"
#include "launch.hpp"

namespace cdbm {

namespace {

// out = w_add * add + w_in * E'(g)^T a, and the per-block partial sums of
// w_in * sum_i a_i dE_i/dtau = w_in * sum_i a_i dt (g_i - g_i^eq) / tau^2
// written to tau_part (acc = 0) or added to it (acc = 1).
// The state g is in the storage precision S; adjoint vectors are double.
// A block is 64 cells of one row (blocks numbered along the row, then row by
// row) and four waves.  Waves 0 and 1 form the pointwise part: wave 0 the
// macroscopic state and the tau term, wave 1 the equilibrium transpose,
// shared through LDS.  Then wave w takes velocities w, w + 4, w + 8 and
// w + 12 and reads each velocity's stencils, the state on offsets -3 .. 3
// (for the face selections at -2 .. 2) and the adjoint on -2 .. 2, along x
// and along y, straight from global memory: neighbouring lanes share cache
// lines, and a block meets one barrier.  At 97 vector registers five waves
// fit per SIMD, so a 256^2 grid's 1024 blocks are all resident at once.
constexpr int ARX = 64, ARW = 4;
static_assert(NV % ARW == 0, "every wave takes the same number of velocities");

template <typename S>
__global__ void __launch_bounds__(ARX * ARW) k_stage_adjoint(const S* __restrict__ g,
                                                             const double* __restrict__ a,
                                                             const double* __restrict__ add,
                                                             double* __restrict__ out,
                                                             double w_in, double w_add,
                                                             KParams K,
                                                             double* __restrict__ tau_part,
                                                             int acc) {
    __shared__ double Mq[8][ARX];   // rho, u_x, u_y, T, then q
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nx = K.nx, ny = K.ny;
    const int bxn = (nx + ARX - 1) / ARX;
    const int x = (int)(blockIdx.x % bxn) * ARX + lane, y = (int)(blockIdx.x / bxn);
    const int64_t cells = (int64_t)nx * ny;
    const bool inside = x < nx;
    const int64_t c = (int64_t)y * nx + x;

    // pointwise part, from the parity transforms pg = P g and pa = P a
    // (P P^T = k I per group, k = 2 axis, 4 diagonal): with h the parity form
    // of f^eq (f^eq = P^T h), a . (g - f^eq) = pa . (pg / k - h).  Each wave
    // loads what it needs, so that wave 1 holds pg only until the moments
    // (this keeps the kernel at 97 registers).
    double tpart = 0.0;
    if (w == 0 && inside) {
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
        Mq[0][lane] = m.rho;
        Mq[1][lane] = m.ux;
        Mq[2][lane] = m.uy;
        Mq[3][lane] = m.T;
    } else if (w == 1 && inside) {
        Macro m;
        {
            Parity pg;
            double v[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) v[i] = (double)g[i * cells + c];
            to_parity(v, pg);
            m = macro_from_parity(pg, K, K.inv_a);
        }
        __builtin_amdgcn_sched_barrier(0);
        Parity pa;
        {
            double v[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) v[i] = a[i * cells + c];
            to_parity(v, pa);
        }
        const Quad q = equilibrium_vjp_q_parity(m, K, K.a, pa);
        Mq[4][lane] = q.rho;
        Mq[5][lane] = q.ux;
        Mq[6][lane] = q.uy;
        Mq[7][lane] = q.T;
    }
    __syncthreads();
    if (w == 0) {   // the block's tau partial, summed in a fixed order
        double v = tpart * w_in;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) tau_part[blockIdx.x] = acc ? tau_part[blockIdx.x] + v : v;
    }
    if (!inside) return;
    const Macro m{Mq[0][lane], Mq[1][lane], Mq[2][lane], Mq[3][lane]};
    const Quad q{Mq[4][lane], Mq[5][lane], Mq[6][lane], Mq[7][lane]};

    // stencil positions, offsets -3 .. 3, through the boundary conditions;
    // the adjoint is zero at zero-gradient ghosts
    const int64_t row = (int64_t)y * nx;
    int xs[7], ys[7];
    bool xg[7], yg[7];
#pragma unroll
    for (int d = -3; d <= 3; ++d) {
        xs[d + 3] = wrap_or_clamp(x + d, nx, K.bcx);
        ys[d + 3] = wrap_or_clamp(y + d, ny, K.bcy);
        xg[d + 3] = K.bcx != CDBM_PERIODIC && (x + d < 0 || x + d >= nx);
        yg[d + 3] = K.bcy != CDBM_PERIODIC && (y + d < 0 || y + d >= ny);
    }
#pragma unroll 1
    for (int j = 0; j < NV / ARW; ++j) {
        const int i = w + ARW * j;
        const int sx = SX[i], sy = SY[i];
        const S* gi = g + i * cells;
        const double* ai = a + i * cells;
        const S fc = gi[c];
        const double ac = ai[c];
        double adv = 0.0;
        if (sx != 0) {
            S F[7];
            RegSel Sl;
            RegLine A;
#pragma unroll
            for (int d = 0; d < 7; ++d) F[d] = d == 3 ? fc : gi[row + xs[d]];
#pragma unroll
            for (int d = 0; d < 5; ++d) {
                Sl.c[d] = face_code<S>(F[d], F[d + 1], F[d + 2]);
                A.v[d] = d == 2 ? ac : (xg[d + 1] ? 0.0 : ai[row + xs[d + 1]]);
            }
            if (sx > 0)
                adv += K.cx[i] * nnd_transpose<true>(Sl, A, 0, x, nx, K.bcx);
            else
                adv += K.cx[i] * nnd_transpose<false>(Sl, A, 0, x, nx, K.bcx);
        }
        if (sy != 0) {
            S F[7];
            RegSel Sl;
            RegLine A;
#pragma unroll
            for (int d = 0; d < 7; ++d) F[d] = d == 3 ? fc : gi[(int64_t)ys[d] * nx + x];
#pragma unroll
            for (int d = 0; d < 5; ++d) {
                Sl.c[d] = face_code<S>(F[d], F[d + 1], F[d + 2]);
                A.v[d] = d == 2 ? ac : (yg[d + 1] ? 0.0 : ai[(int64_t)ys[d + 1] * nx + x]);
            }
            if (sy > 0)
                adv += K.cy[i] * nnd_transpose<true>(Sl, A, 0, y, ny, K.bcy);
            else
                adv += K.cy[i] * nnd_transpose<false>(Sl, A, 0, y, ny, K.bcy);
        }
        const double ceq = moments_vjp_k(m, K, K.a, q, i);
        double v = ac + adv - K.z * (ac - ceq);
        v *= w_in;
        if (w_add != 0.0) v = fma(w_add, add[i * cells + c], v);
        out[i * cells + c] = v;
    }
}

// Sum of part[i], part[i + step], ... (i < n) over the 1024 threads of a
// block, thread t starting at its own i, in a fixed order: up to four loads
// in flight per thread, each wave's 64 sums by shuffles, then the 16 wave
// sums by the first wave.  The result is valid in thread 0.  With clear,
// every element read is set to zero.
__device__ __forceinline__ double block_sum_1024(double* __restrict__ part, int64_t i,
                                                 int64_t step, int64_t n, bool clear) {
    __shared__ double red[16];
    double s = 0.0;
    for (; i + 3 * step < n; i += 4 * step) {
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = part[i + k * step];
        if (clear) {
#pragma unroll
            for (int k = 0; k < 4; ++k) part[i + k * step] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) s += v[k];
    }
    for (; i < n; i += step) {
        s += part[i];
        if (clear) part[i] = 0.0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < 64) {
        t = threadIdx.x < 16 ? red[threadIdx.x] : 0.0;
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) t += __shfl_xor(t, o);
    }
    return t;
}

// dst[0] += scale * sum_b part[b] by one block (part cleared with clear).
__global__ void __launch_bounds__(1024) k_accumulate(double* __restrict__ part, int64_t n,
                                                     double scale, double* __restrict__ dst,
                                                     int clear) {
    const double t = block_sum_1024(part, threadIdx.x, 1024, n, clear != 0);
    if (threadIdx.x == 0) dst[0] += scale * t;
}

// out[k] = sum of part[b] over b = 1024 k + t + j 1024 gridDim.x: the first
// pass of a two-pass sum of many partials.
__global__ void __launch_bounds__(1024) k_partial_sum(double* __restrict__ part, int64_t n,
                                                      double* __restrict__ out, int clear) {
    const double t = block_sum_1024(part, (int64_t)blockIdx.x * 1024 + threadIdx.x,
                                    (int64_t)gridDim.x * 1024, n, clear != 0);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
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
    return (int)(blocks_for(K.nx, ARX) * (unsigned)K.ny);
}

template <typename S>
hipError_t launch_stage_adjoint(const void* g, const void* a, const void* add, void* out,
                                double* tau_part, bool tau_add, double w_in, double w_add,
                                const KParams& K, hipStream_t st) {
    hipLaunchKernelGGL(k_stage_adjoint<S>, dim3(stage_adjoint_blocks(K)), dim3(ARX * ARW), 0, st,
                       (const S*)g, (const double*)a, (const double*)add, (double*)out, w_in,
                       w_add, K, tau_part, tau_add ? 1 : 0);
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

hipError_t launch_accumulate_scalar(double* part, int n, double* scratch, double scale,
                                    double* dst, bool clear, hipStream_t st) {
    if (n > ACCUMULATE_ONE_PASS) {
        hipLaunchKernelGGL(k_partial_sum, dim3(ACCUMULATE_BLOCKS), dim3(1024), 0, st, part,
                           (int64_t)n, scratch, clear ? 1 : 0);
        part = scratch;
        n = ACCUMULATE_BLOCKS;
        clear = false;
    }
    hipLaunchKernelGGL(k_accumulate, dim3(1), dim3(1024), 0, st, part, (int64_t)n, scale, dst,
                       clear ? 1 : 0);
    return hipGetLastError();
}

#define CDBM_INSTANTIATE(S)                                                                      \
    template hipError_t launch_stage_adjoint<S>(const void*, const void*, const void*, void*,   \
                                                double*, bool, double, double, const KParams&,  \
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
