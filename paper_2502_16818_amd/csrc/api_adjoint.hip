// C ABI of the reverse-mode products (include/cdbm.h).
//
// One step is F(f) = f/2 + E(E(f))/2 with the stage E(g) = g + dt L(g).
// With lam' = lam^{n+1} and f1 = E(f):
//   mu    = E'(f1)^T lam' / 2
//   lam^n = lam' / 2 + E'(f)^T mu
//   dL/dtau += lam' . dE/dtau(f1) / 2 + mu . dE/dtau(f)
// f1 is recomputed from f (the unfused stage kernel) into the handle's stage
// buffer, or supplied by the caller (cdbm_step_adjoint_stage); mu lives in a
// second handle-owned buffer.  The two stage adjoints
// leave their per-block tau partials side by side, summed by one launch.  Adjoint vectors are
// double in both precision forms: for a loss of the density alone lam_i is
// close to one value for all i, and the gradient with respect to u and T is
// carried by its small deviations, which FP32 storage would round away.
#include <hip/hip_runtime.h>

#include "../../include/cdbm.h"
#include "api_internal.hpp"
#include "launch.hpp"

using namespace cdbm;

namespace {

// f1: the first stage of the step, or nullptr to recompute it into the
// handle's stage buffer.
template <typename S>
int step_adjoint_impl(cdbm_handle* h, const void* f_n, const void* f1, const void* lam_np1,
                      void* lam_n, double* dtau, hipStream_t st) {
    const KParams& K = h->k;
    const int nb = stage_adjoint_blocks(K);
    hipError_t e = hipSuccess;
    if (!f1) {
        e = launch_stage<S>(f_n, nullptr, h->stage, false, K, h->kdev, st);
        if (e != hipSuccess) return hip_fail(e, "stage recompute launch");
        f1 = h->stage;
    }
    // without dtau, both stages add their block partials to the handle's
    // accumulator (cdbm_tau_collect sums it); else they write them side by
    // side and one fixed-order sum adds them to dtau
    const bool defer = dtau == nullptr;
    double* part2 = defer ? h->tau_acc : h->tau_part;
    double* part1 = defer ? h->tau_acc : h->tau_part + nb;
    e = launch_stage_adjoint<S>(f1, lam_np1, nullptr, h->lam_mid, part2, defer, 0.5, 0.0, K, st);
    if (e != hipSuccess) return hip_fail(e, "stage adjoint launch");
    e = launch_stage_adjoint<S>(f_n, h->lam_mid, lam_np1, lam_n, part1, defer, 1.0, 0.5, K, st);
    if (e != hipSuccess) return hip_fail(e, "stage adjoint launch");
    if (defer) return CDBM_OK;
    e = launch_accumulate_scalar(h->tau_part, 2 * nb, h->tau_part + 2 * nb, 1.0, dtau, false, st);
    if (e != hipSuccess) return hip_fail(e, "tau accumulation launch");
    return CDBM_OK;
}

// Do [a, a + an) and [b, b + bn) intersect?
bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + bn && y < x + an;
}

// Checks and buffers shared by both step adjoints (f1 may be nullptr).
int step_adjoint_entry(cdbm_handle* h, const void* f_n, const void* f1, const void* lam_np1,
                       void* lam_n, double* dL_dtau, void* stream) {
    const size_t lbytes = sizeof(double) * (size_t)NV * (size_t)h->cells;
    if (overlaps(lam_n, lbytes, f_n, h->fbytes) || overlaps(lam_n, lbytes, lam_np1, lbytes))
        return fail(CDBM_EINVAL, "lam_n overlaps f_n or lam_np1");
    if (f1 && overlaps(lam_n, lbytes, f1, h->fbytes))
        return fail(CDBM_EINVAL, "lam_n overlaps f1");
    int rc = check_device(h);
    if (rc != CDBM_OK) return rc;
    if (!f1 && (rc = ensure_buffer(h, &h->stage)) != CDBM_OK) return rc;
    if (!h->lam_mid &&
        hipMalloc(&h->lam_mid, sizeof(double) * (size_t)NV * (size_t)h->cells) != hipSuccess) {
        h->lam_mid = nullptr;
        return fail(CDBM_ENOMEM, "hipMalloc of the adjoint buffer failed");
    }
    hipStream_t st = (hipStream_t)stream;
    return mixed(h) ? step_adjoint_impl<float>(h, f_n, f1, lam_np1, lam_n, dL_dtau, st)
                    : step_adjoint_impl<double>(h, f_n, f1, lam_np1, lam_n, dL_dtau, st);
}

}  // namespace

extern "C" {

int cdbm_step_adjoint(cdbm_handle* h, const void* f_n, const void* lam_np1, void* lam_n,
                      double* dL_dtau, void* stream) {
    if (!h || !f_n || !lam_np1 || !lam_n) return fail(CDBM_EINVAL, "null argument");
    if (comp(h)) return fail(CDBM_EINVAL, "the adjoint entry points do not take CDBM_MIXED_COMP");
    return step_adjoint_entry(h, f_n, nullptr, lam_np1, lam_n, dL_dtau, stream);
}

int cdbm_step_adjoint_stage(cdbm_handle* h, const void* f_n, const void* f1,
                            const void* lam_np1, void* lam_n, double* dL_dtau, void* stream) {
    if (!h || !f_n || !f1 || !lam_np1 || !lam_n) return fail(CDBM_EINVAL, "null argument");
    if (comp(h)) return fail(CDBM_EINVAL, "the adjoint entry points do not take CDBM_MIXED_COMP");
    return step_adjoint_entry(h, f_n, f1, lam_np1, lam_n, dL_dtau, stream);
}

int cdbm_tau_collect(cdbm_handle* h, double* dL_dtau, void* stream) {
    if (!h || !dL_dtau) return fail(CDBM_EINVAL, "null argument");
    if (comp(h)) return fail(CDBM_EINVAL, "the adjoint entry points do not take CDBM_MIXED_COMP");
    int rc = check_device(h);
    if (rc != CDBM_OK) return rc;
    const int nb = stage_adjoint_blocks(h->k);
    hipError_t e = launch_accumulate_scalar(h->tau_acc, nb, h->tau_part + 2 * nb, 1.0, dL_dtau,
                                            true, (hipStream_t)stream);
    return e == hipSuccess ? CDBM_OK : hip_fail(e, "tau collect launch");
}

int cdbm_init_adjoint(cdbm_handle* h, const double* rho, const double* ux, const double* uy,
                      const double* T, const void* lam_f0, double* g_rho, double* g_ux,
                      double* g_uy, double* g_T, void* stream) {
    if (!h || !rho || !ux || !uy || !T || !lam_f0 || !g_rho || !g_ux || !g_uy || !g_T)
        return fail(CDBM_EINVAL, "null argument");
    if (comp(h)) return fail(CDBM_EINVAL, "the adjoint entry points do not take CDBM_MIXED_COMP");
    int rc = check_device(h);
    if (rc != CDBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e =
        mixed(h) ? launch_init_adjoint<float>(rho, ux, uy, T, lam_f0, g_rho, g_ux, g_uy, g_T, h->k, st)
                 : launch_init_adjoint<double>(rho, ux, uy, T, lam_f0, g_rho, g_ux, g_uy, g_T, h->k,
                                               st);
    return e == hipSuccess ? CDBM_OK : hip_fail(e, "init adjoint launch");
}

int cdbm_moments_adjoint(cdbm_handle* h, const void* f, const double* g_rho, const double* g_ux,
                         const double* g_uy, const double* g_T, void* lam_f, void* stream) {
    if (!h || !f || !g_rho || !g_ux || !g_uy || !g_T || !lam_f)
        return fail(CDBM_EINVAL, "null argument");
    if (comp(h)) return fail(CDBM_EINVAL, "the adjoint entry points do not take CDBM_MIXED_COMP");
    if (overlaps(lam_f, sizeof(double) * (size_t)NV * (size_t)h->cells, f, h->fbytes))
        return fail(CDBM_EINVAL, "lam_f overlaps f");
    int rc = check_device(h);
    if (rc != CDBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = mixed(h)
                       ? launch_moments_adjoint<float>(f, g_rho, g_ux, g_uy, g_T, lam_f, h->k, st)
                       : launch_moments_adjoint<double>(f, g_rho, g_ux, g_uy, g_T, lam_f, h->k, st);
    return e == hipSuccess ? CDBM_OK : hip_fail(e, "moments adjoint launch");
}

}  // extern "C"
