// C ABI of the CDBM library (include/cdbm.h): handle lifetime, argument
// checks, buffer ping-pong, graph capture of the step loop.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cdbm.h"
#include "api_internal.hpp"
#include "launch.hpp"
#include "model.hpp"

using cdbm::KParams;

namespace cdbm {

namespace {
thread_local std::string g_err;
constexpr int GRAPH_STEPS = 32;   // steps per captured graph (an even number)
}  // namespace

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    g_err = buf;
    return CDBM_EHIP;
}

int check_device(const cdbm_handle* h) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != h->device) return fail(CDBM_EINVAL, "handle was created on another device");
    return CDBM_OK;
}

int ensure_buffer(cdbm_handle* h, void** buf) {
    if (*buf) return CDBM_OK;
    hipError_t e = hipMalloc(buf, h->fbytes);
    if (e != hipSuccess) {
        *buf = nullptr;
        return fail(CDBM_ENOMEM, "hipMalloc of an f-sized buffer failed");
    }
    return CDBM_OK;
}

const char* last_error() { return g_err.c_str(); }

int check_fields_range(int* flag, const double* rho, const double* ux, const double* uy,
                       const double* T, int64_t cells, hipStream_t st) {
    if (!rho || !ux || !uy || !T) return fail(CDBM_EINVAL, "null field pointer");
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), st);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    e = launch_check_fields(rho, ux, uy, T, cells, flag, st);
    if (e != hipSuccess) return hip_fail(e, "field check launch");
    int bad = 0;
    e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (bad) return fail(CDBM_ENONPHYS, "rho <= 0, T <= 0 or a non-finite value in the fields");
    return CDBM_OK;
}

void StepGraph::drop(Entry& en) {
    if (en.exec) {
        if (en.launched && en.done) (void)hipEventSynchronize(en.done);
        (void)hipGraphExecDestroy(en.exec);
    }
    en.exec = nullptr;
    en.out = nullptr;
    en.launched = false;
}

void StepGraph::release() {
    for (Entry& en : slot) {
        drop(en);
        if (en.done) (void)hipEventDestroy(en.done);
        en.done = nullptr;
    }
    if (cap) (void)hipStreamDestroy(cap);
    cap = nullptr;
}

namespace {

// The graph entry that replays GRAPH_STEPS steps into `fout`, captured on
// first use.
int graph_for(StepFn fn, const void* ctx, void* fout, void* scratch, StepGraph& graph,
              StepGraph::Entry** out) {
    for (StepGraph::Entry& en : graph.slot)
        if (en.exec && en.out == fout) {
            *out = &en;
            return CDBM_OK;
        }
    StepGraph::Entry& en = graph.slot[graph.next];
    graph.next ^= 1;
    graph.drop(en);
    hipError_t e;
    if (!graph.cap) {
        e = hipStreamCreateWithFlags(&graph.cap, hipStreamNonBlocking);
        if (e != hipSuccess) {
            graph.cap = nullptr;
            return hip_fail(e, "hipStreamCreateWithFlags");
        }
    }
    if (!en.done) {
        e = hipEventCreateWithFlags(&en.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            en.done = nullptr;
            return hip_fail(e, "hipEventCreateWithFlags");
        }
    }
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(graph.cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = hipSuccess;
    for (int s = 0; s < GRAPH_STEPS && le == hipSuccess; ++s)
        le = (s % 2 == 0) ? fn(ctx, fout, scratch, graph.cap) : fn(ctx, scratch, fout, graph.cap);
    e = hipStreamEndCapture(graph.cap, &g);
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le != hipSuccess ? le : e, "step graph capture");
    }
    e = hipGraphInstantiate(&en.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        en.exec = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    en.out = fout;
    *out = &en;
    return CDBM_OK;
}

}  // namespace

int run_steps(StepFn fn, const void* ctx, const void* fin, void* fout, void* scratch, int nsteps,
              hipStream_t st, StepGraph& graph) {
    int remaining = nsteps;
    hipError_t e;
    if (nsteps % 2 == 1) {
        e = fn(ctx, fin, fout, st);
        if (e != hipSuccess) return hip_fail(e, "step launch");
        --remaining;
    } else {
        e = fn(ctx, fin, scratch, st);
        if (e == hipSuccess) e = fn(ctx, scratch, fout, st);
        if (e != hipSuccess) return hip_fail(e, "step launch");
        remaining -= 2;
    }
    // remaining is even and the state is in fout
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool can_graph =
        st == nullptr || (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone);
    if (can_graph && remaining >= GRAPH_STEPS) {
        StepGraph::Entry* en = nullptr;
        int rc = graph_for(fn, ctx, fout, scratch, graph, &en);
        if (rc != CDBM_OK) return rc;
        while (remaining >= GRAPH_STEPS) {
            e = hipGraphLaunch(en->exec, st);
            if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
            en->launched = true;
            remaining -= GRAPH_STEPS;
        }
        e = hipEventRecord(en->done, st);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    while (remaining > 0) {
        e = fn(ctx, fout, scratch, st);
        if (e == hipSuccess) e = fn(ctx, scratch, fout, st);
        if (e != hipSuccess) return hip_fail(e, "step launch");
        remaining -= 2;
    }
    return CDBM_OK;
}

namespace {

// With CDBM_STEP_AUTO, grids of up to this many cells take the step as two
// single-stage launches (f^(1) through the handle's stage buffer): one cell
// per thread fills the chip, where the fused step has too few rows per block
// to hide its per-iteration latency (measured crossovers: about 700 x 700
// cells in the mixed form, about 560 x 560 in FP64).
constexpr int64_t SPLIT_STEP_CELLS_MIXED = int64_t(1) << 19;   // 724 x 724
constexpr int64_t SPLIT_STEP_CELLS_FP64 = int64_t(1) << 18;    // 512 x 512

hipError_t step_once(const cdbm_handle* h, const void* fin, void* fout, hipStream_t st) {
    if (comp(h)) {
        hipError_t e = launch_stage_comp(fin, nullptr, h->stage, false, h->k, h->kdev, st);
        if (e != hipSuccess) return e;
        return launch_stage_comp(h->stage, fin, fout, true, h->k, h->kdev, st);
    }
    if (h->split) {
        hipError_t e = mixed(h) ? launch_stage<float>(fin, nullptr, h->stage, false, h->k, h->kdev, st)
                                : launch_stage<double>(fin, nullptr, h->stage, false, h->k, h->kdev, st);
        if (e != hipSuccess) return e;
        return mixed(h) ? launch_stage<float>(h->stage, fin, fout, true, h->k, h->kdev, st)
                        : launch_stage<double>(h->stage, fin, fout, true, h->k, h->kdev, st);
    }
    return mixed(h) ? launch_step_fused<float>(fin, fout, h->k, h->kdev, st)
                    : launch_step_fused<double>(fin, fout, h->k, h->kdev, st);
}

int check_fields(cdbm_handle* h, const double* rho, const double* ux, const double* uy,
                 const double* T, hipStream_t st) {
    return check_fields_range(h->flag, rho, ux, uy, T, h->cells, st);
}

hipError_t step_single(const void* ctx, const void* fin, void* fout, hipStream_t st) {
    return step_once((const cdbm_handle*)ctx, fin, fout, st);
}

// two time steps in one launch (CDBM_STEP_FUSED2)
hipError_t step_pair(const void* ctx, const void* fin, void* fout, hipStream_t st) {
    const cdbm_handle* h = (const cdbm_handle*)ctx;
    return launch_step2_fused(fin, fout, h->k, h->kdev, st);
}

}  // namespace
}  // namespace cdbm

using namespace cdbm;

extern "C" {

const char* cdbm_last_error(void) { return cdbm::last_error(); }

int cdbm_create(const cdbm_params* p, cdbm_handle** out) {
    if (!p || !out) return fail(CDBM_EINVAL, "null argument");
    *out = nullptr;
    auto* h = new (std::nothrow) cdbm_handle();
    if (!h) return fail(CDBM_ENOMEM, "host allocation failed");
    h->p = *p;
    std::string err;
    int rc = cdbm::build_params(*p, h->k, err);
    if (rc != CDBM_OK) {
        delete h;
        return fail(rc, err);
    }
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipGetDevice");
    }
    h->cells = (int64_t)p->nx * p->ny;
    h->elem = (mixed(h) || comp(h)) ? sizeof(float) : sizeof(double);
    h->fbytes = (size_t)state_planes(p->precision) * (size_t)h->cells * h->elem;
    // tau partials of the two stage adjoints of a step, side by side, then
    // room for the second-level sums of a two-pass accumulation
    const int tau_blocks = 2 * stage_adjoint_blocks(h->k) + ACCUMULATE_BLOCKS;
    h->split = p->step_form == CDBM_STEP_SPLIT || comp(h) ||
               (p->step_form == CDBM_STEP_AUTO &&
                h->cells <= (mixed(h) ? SPLIT_STEP_CELLS_MIXED : SPLIT_STEP_CELLS_FP64));
    h->two = p->step_form == CDBM_STEP_FUSED2;
    if (ensure_buffer(h, &h->scratch) != CDBM_OK ||
        ((h->split || h->two) && ensure_buffer(h, &h->stage) != CDBM_OK) ||
        hipMalloc(&h->partials, sizeof(double) * 4 * REDUCE_BLOCKS) != hipSuccess ||
        hipMalloc(&h->tau_part, sizeof(double) * tau_blocks) != hipSuccess ||
        hipMalloc(&h->tau_acc, sizeof(double) * stage_adjoint_blocks(h->k)) != hipSuccess ||
        hipMalloc(&h->flag, sizeof(int)) != hipSuccess ||
        hipMalloc(&h->kdev, sizeof(KParams)) != hipSuccess) {
        cdbm_destroy(h);
        return fail(CDBM_ENOMEM, "device allocation failed");
    }
    e = hipMemcpy(h->kdev, &h->k, sizeof(KParams), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemset(h->tau_acc, 0, sizeof(double) * stage_adjoint_blocks(h->k));
    if (e != hipSuccess) {
        cdbm_destroy(h);
        return hip_fail(e, "copying the run constants / clearing the tau accumulator");
    }
    *out = h;
    return CDBM_OK;
}

int cdbm_destroy(cdbm_handle* h) {
    if (!h) return CDBM_OK;
    (void)hipDeviceSynchronize();
    h->graph.release();
    if (h->scratch) (void)hipFree(h->scratch);
    if (h->stage) (void)hipFree(h->stage);
    if (h->lam_mid) (void)hipFree(h->lam_mid);
    if (h->partials) (void)hipFree(h->partials);
    if (h->tau_part) (void)hipFree(h->tau_part);
    if (h->tau_acc) (void)hipFree(h->tau_acc);
    if (h->flag) (void)hipFree(h->flag);
    if (h->kdev) (void)hipFree(h->kdev);
    delete h;
    return CDBM_OK;
}

int cdbm_get_params(const cdbm_handle* h, cdbm_params* out) {
    if (!h || !out) return fail(CDBM_EINVAL, "null argument");
    *out = h->p;
    return CDBM_OK;
}

int cdbm_init(cdbm_handle* h, const double* rho, const double* ux, const double* uy,
              const double* T, void* f_out, void* stream) {
    if (!h || !f_out) return fail(CDBM_EINVAL, "null argument");
    int rc = check_device(h);
    if (rc != CDBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    rc = check_fields(h, rho, ux, uy, T, st);
    if (rc != CDBM_OK) return rc;
    hipError_t e = comp(h)    ? cdbm::launch_init_comp(rho, ux, uy, T, f_out, h->k, st)
                   : mixed(h) ? cdbm::launch_init<float>(rho, ux, uy, T, f_out, h->k, st)
                              : cdbm::launch_init<double>(rho, ux, uy, T, f_out, h->k, st);
    return e == hipSuccess ? CDBM_OK : hip_fail(e, "init launch");
}

int cdbm_step(cdbm_handle* h, const void* f_in, void* f_out, int32_t nsteps, void* stream) {
    if (!h || !f_in || !f_out) return fail(CDBM_EINVAL, "null argument");
    if (nsteps < 0) return fail(CDBM_EINVAL, "nsteps must be >= 0");
    const char* a = (const char*)f_in;
    const char* b = (const char*)f_out;
    if (a < b + h->fbytes && b < a + h->fbytes) return fail(CDBM_EINVAL, "f_in and f_out overlap");
    int rc = check_device(h);
    if (rc != CDBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (nsteps == 0) {
        hipError_t e = hipMemcpyAsync(f_out, f_in, h->fbytes, hipMemcpyDeviceToDevice, st);
        return e == hipSuccess ? CDBM_OK : hip_fail(e, "hipMemcpyAsync");
    }
    if (h->two) {
        // pairs of steps per launch; an odd last step runs fused, from the
        // pairs' result in the handle's stage buffer
        const int pairs = nsteps / 2;
        if (nsteps % 2 == 0) return run_steps(step_pair, h, f_in, f_out, h->scratch, pairs, st, h->graph);
        const void* src = f_in;
        if (pairs > 0) {
            rc = run_steps(step_pair, h, f_in, h->stage, h->scratch, pairs, st, h->graph);
            if (rc != CDBM_OK) return rc;
            src = h->stage;
        }
        hipError_t e = launch_step_fused<float>(src, f_out, h->k, h->kdev, st);
        return e == hipSuccess ? CDBM_OK : hip_fail(e, "step launch");
    }
    return run_steps(step_single, h, f_in, f_out, h->scratch, nsteps, st, h->graph);
}

int cdbm_step_keep_stage(cdbm_handle* h, const void* f_in, void* f1_out, void* f_out,
                         void* stream) {
    if (!h || !f_in || !f1_out || !f_out) return fail(CDBM_EINVAL, "null argument");
    if (comp(h)) return fail(CDBM_EINVAL, "cdbm_step_keep_stage does not take CDBM_MIXED_COMP");
    const char* a = (const char*)f_in;
    const char* b = (const char*)f1_out;
    const char* c = (const char*)f_out;
    const size_t n = h->fbytes;
    if ((a < b + n && b < a + n) || (a < c + n && c < a + n) || (b < c + n && c < b + n))
        return fail(CDBM_EINVAL, "f_in, f1_out and f_out must not overlap");
    int rc = check_device(h);
    if (rc != CDBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = mixed(h) ? launch_stage<float>(f_in, nullptr, f1_out, false, h->k, h->kdev, st)
                            : launch_stage<double>(f_in, nullptr, f1_out, false, h->k, h->kdev, st);
    if (e == hipSuccess)
        e = mixed(h) ? launch_stage<float>(f1_out, f_in, f_out, true, h->k, h->kdev, st)
                     : launch_stage<double>(f1_out, f_in, f_out, true, h->k, h->kdev, st);
    return e == hipSuccess ? CDBM_OK : hip_fail(e, "stage launch");
}

int cdbm_moments(cdbm_handle* h, const void* f, double* rho, double* ux, double* uy, double* T,
                 void* stream) {
    if (!h || !f || !rho || !ux || !uy || !T) return fail(CDBM_EINVAL, "null argument");
    int rc = check_device(h);
    if (rc != CDBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = comp(h)    ? cdbm::launch_moments_comp(f, rho, ux, uy, T, h->k, st)
                   : mixed(h) ? cdbm::launch_moments<float>(f, rho, ux, uy, T, h->k, st)
                              : cdbm::launch_moments<double>(f, rho, ux, uy, T, h->k, st);
    return e == hipSuccess ? CDBM_OK : hip_fail(e, "moments launch");
}

namespace {
int tne_common(cdbm_handle* h, const void* f, double* out12, bool raw, void* stream) {
    if (!h || !f || !out12) return fail(CDBM_EINVAL, "null argument");
    int rc = check_device(h);
    if (rc != CDBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = comp(h)    ? cdbm::launch_tne_comp(f, out12, raw, h->k, st)
                   : mixed(h) ? cdbm::launch_tne<float>(f, out12, raw, h->k, st)
                              : cdbm::launch_tne<double>(f, out12, raw, h->k, st);
    return e == hipSuccess ? CDBM_OK : hip_fail(e, "tne launch");
}
}  // namespace

int cdbm_tne(cdbm_handle* h, const void* f, double* out12, void* stream) {
    return tne_common(h, f, out12, false, stream);
}

int cdbm_tne_raw(cdbm_handle* h, const void* f, double* out12, void* stream) {
    return tne_common(h, f, out12, true, stream);
}

int cdbm_conserved_totals(cdbm_handle* h, const void* f, double* out4, void* stream) {
    if (!h || !f || !out4) return fail(CDBM_EINVAL, "null argument");
    int rc = check_device(h);
    if (rc != CDBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e =
        comp(h)    ? cdbm::launch_totals_comp(f, h->partials, REDUCE_BLOCKS, out4, h->k, st)
        : mixed(h) ? cdbm::launch_totals<float>(f, h->partials, REDUCE_BLOCKS, out4, h->k, st)
                   : cdbm::launch_totals<double>(f, h->partials, REDUCE_BLOCKS, out4, h->k, st);
    return e == hipSuccess ? CDBM_OK : hip_fail(e, "totals launch");
}

}  // extern "C"
