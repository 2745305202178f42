// C ABI of the batched ensemble (include/cdbm.h): independent grids with
// their own sizes, gamma, tau, dt, spacings and boundary conditions, sharing
// one velocity set, advanced by one persistent launch per step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/cdbm.h"
#include "api_internal.hpp"
#include "launch.hpp"
#include "step_fused.hpp"

using namespace cdbm;

struct cdbm_batch {
    std::vector<cdbm_params> p;
    std::vector<KParams> k;
    std::vector<int64_t> off;
    int device = 0;
    int precision = CDBM_FP64;
    size_t elem = 8;
    int64_t total_elems = 0;    // extent of the batch buffers (elements)
    KParams* d_k = nullptr;
    int64_t* d_off = nullptr;
    int64_t* d_work = nullptr;
    int* flag = nullptr;
    void* scratch = nullptr;
    int nblocks = 1;
    bool chunked = false;   // every width and offset is a multiple of the 16-byte chunk
    StepGraph graph;
};

namespace {

void release(cdbm_batch* b) {
    b->graph.release();
    if (b->d_k) (void)hipFree(b->d_k);
    if (b->d_off) (void)hipFree(b->d_off);
    if (b->d_work) (void)hipFree(b->d_work);
    if (b->flag) (void)hipFree(b->flag);
    if (b->scratch) (void)hipFree(b->scratch);
    delete b;
}

hipError_t batch_step_once(const void* ctx, const void* fin, void* fout, hipStream_t st) {
    const cdbm_batch* b = (const cdbm_batch*)ctx;
    const int n = (int)b->p.size();
    return b->precision == CDBM_MIXED
               ? launch_batch_step<float>(fin, fout, b->d_k, b->d_off, b->d_work, n, b->nblocks,
                                          b->chunked, st)
               : launch_batch_step<double>(fin, fout, b->d_k, b->d_off, b->d_work, n, b->nblocks,
                                           b->chunked, st);
}

int check_batch_device(const cdbm_batch* b) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != b->device) return fail(CDBM_EINVAL, "batch was created on another device");
    return CDBM_OK;
}

}  // namespace

extern "C" {

int cdbm_batch_create(const cdbm_params* per_grid, int32_t ngrids, const int64_t* f_offsets,
                      cdbm_batch** out) {
    if (!per_grid || !f_offsets || !out) return fail(CDBM_EINVAL, "null argument");
    *out = nullptr;
    if (ngrids < 1 || ngrids > (1 << 20)) return fail(CDBM_EINVAL, "ngrids out of range");
    auto* b = new (std::nothrow) cdbm_batch();
    if (!b) return fail(CDBM_ENOMEM, "host allocation failed");
    b->p.assign(per_grid, per_grid + ngrids);
    b->k.resize(ngrids);
    b->off.assign(f_offsets, f_offsets + ngrids);
    b->precision = per_grid[0].precision;
    char buf[160];
    for (int g = 0; g < ngrids; ++g) {
        const cdbm_params& q = per_grid[g];
        std::string err;
        int rc = build_params(q, b->k[g], err);
        if (rc != CDBM_OK) {
            std::snprintf(buf, sizeof buf, "grid %d: ", g);
            delete b;
            return fail(rc, buf + err);
        }
        if (std::memcmp(q.v, per_grid[0].v, sizeof q.v) != 0 ||
            std::memcmp(q.eta, per_grid[0].eta, sizeof q.eta) != 0 ||
            q.precision != per_grid[0].precision) {
            std::snprintf(buf, sizeof buf,
                          "grid %d: v, eta and precision must be the same for every grid", g);
            delete b;
            return fail(CDBM_EINVAL, buf);
        }
        if (f_offsets[g] < 0) {
            delete b;
            return fail(CDBM_EINVAL, "negative f offset");
        }
    }
    // the grids' blocks must not overlap
    std::vector<int> order(ngrids);
    for (int g = 0; g < ngrids; ++g) order[g] = g;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return f_offsets[x] < f_offsets[y]; });
    int64_t end = 0;
    for (int idx = 0; idx < ngrids; ++idx) {
        const int g = order[idx];
        const int64_t sz = (int64_t)NV * per_grid[g].nx * per_grid[g].ny;
        if (f_offsets[g] < end) {
            delete b;
            return fail(CDBM_EINVAL, "f blocks of the grids overlap");
        }
        end = f_offsets[g] + sz;
    }
    b->total_elems = end;
    b->elem = b->precision == CDBM_MIXED ? sizeof(float) : sizeof(double);

    std::vector<int64_t> work(ngrids + 1, 0);
    int64_t strip_rows = 0;
    for (int g = 0; g < ngrids; ++g) {
        const int tx = strip_width(b->precision);
        const int64_t strips = (per_grid[g].nx + tx - 1) / tx;
        strip_rows += strips * per_grid[g].ny;
        work[g + 1] = work[g] + strips * (per_grid[g].ny + BATCH_FILL);
    }
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "hipGetDevice");
    }
    if (hipMalloc(&b->d_k, sizeof(KParams) * ngrids) != hipSuccess ||
        hipMalloc(&b->d_off, sizeof(int64_t) * ngrids) != hipSuccess ||
        hipMalloc(&b->d_work, sizeof(int64_t) * (ngrids + 1)) != hipSuccess ||
        hipMalloc(&b->flag, sizeof(int)) != hipSuccess ||
        hipMalloc(&b->scratch, (size_t)b->total_elems * b->elem) != hipSuccess) {
        release(b);
        return fail(CDBM_ENOMEM, "device allocation failed");
    }
    if ((e = hipMemcpy(b->d_k, b->k.data(), sizeof(KParams) * ngrids, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(b->d_off, f_offsets, sizeof(int64_t) * ngrids, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(b->d_work, work.data(), sizeof(int64_t) * (ngrids + 1),
                       hipMemcpyHostToDevice)) != hipSuccess) {
        release(b);
        return hip_fail(e, "hipMemcpy of the batch tables");
    }
    const int64_t cap = (strip_rows + 31) / 32;
    int64_t nb = b->precision == CDBM_MIXED ? batch_blocks<float>() : batch_blocks<double>();
    b->nblocks = (int)std::max<int64_t>(1, std::min(nb, cap));
    // the chunked form of the step (16-byte chunks, 32-bit offsets within a grid)
    const int cw = b->precision == CDBM_MIXED ? 4 : 2;
    const uint64_t esz = b->precision == CDBM_MIXED ? 4 : 8;
    b->chunked = true;
    for (int g = 0; g < ngrids; ++g)
        b->chunked = b->chunked && per_grid[g].nx % cw == 0 && f_offsets[g] % cw == 0 &&
                     (uint64_t)NV * per_grid[g].nx * per_grid[g].ny * esz <= (uint64_t(1) << 32);
    *out = b;
    return CDBM_OK;
}

int cdbm_batch_destroy(cdbm_batch* b) {
    if (!b) return CDBM_OK;
    (void)hipDeviceSynchronize();
    release(b);
    return CDBM_OK;
}

int cdbm_batch_init(cdbm_batch* b, const double* rho, const double* ux, const double* uy,
                    const double* T, void* f_out, void* stream) {
    if (!b || !rho || !ux || !uy || !T || !f_out) return fail(CDBM_EINVAL, "null argument");
    int rc = check_batch_device(b);
    if (rc != CDBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    for (size_t g = 0; g < b->p.size(); ++g) {
        if (b->off[g] % NV != 0)
            return fail(CDBM_EINVAL, "cdbm_batch_init needs f offsets that are multiples of 16");
        const int64_t c0 = b->off[g] / NV;
        const int64_t cells = (int64_t)b->p[g].nx * b->p[g].ny;
        rc = check_fields_range(b->flag, rho + c0, ux + c0, uy + c0, T + c0, cells, st);
        if (rc != CDBM_OK) return rc;
    }
    for (size_t g = 0; g < b->p.size(); ++g) {
        const int64_t c0 = b->off[g] / NV;
        char* dst = (char*)f_out + (size_t)b->off[g] * b->elem;
        hipError_t e =
            b->precision == CDBM_MIXED
                ? launch_init<float>(rho + c0, ux + c0, uy + c0, T + c0, dst, b->k[g], st)
                : launch_init<double>(rho + c0, ux + c0, uy + c0, T + c0, dst, b->k[g], st);
        if (e != hipSuccess) return hip_fail(e, "init launch");
    }
    return CDBM_OK;
}

int cdbm_batch_step(cdbm_batch* b, const void* f_in, void* f_out, int32_t nsteps, void* stream) {
    if (!b || !f_in || !f_out) return fail(CDBM_EINVAL, "null argument");
    if (nsteps < 0) return fail(CDBM_EINVAL, "nsteps must be >= 0");
    const size_t bytes = (size_t)b->total_elems * b->elem;
    const char* x = (const char*)f_in;
    const char* y = (const char*)f_out;
    if (x < y + bytes && y < x + bytes) return fail(CDBM_EINVAL, "f_in and f_out overlap");
    int rc = check_batch_device(b);
    if (rc != CDBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (nsteps == 0) {
        hipError_t e = hipMemcpyAsync(f_out, f_in, bytes, hipMemcpyDeviceToDevice, st);
        return e == hipSuccess ? CDBM_OK : hip_fail(e, "hipMemcpyAsync");
    }
    return run_steps(batch_step_once, b, f_in, f_out, b->scratch, nsteps, st, b->graph);
}

}  // extern "C"
