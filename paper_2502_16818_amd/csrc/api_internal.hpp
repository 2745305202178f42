// Internal declarations shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/cdbm.h"
#include "model.hpp"

namespace cdbm {

// Record an error message for cdbm_last_error() and return `code`.
int fail(int code, const std::string& msg);
// Same for a failed HIP call; returns CDBM_EHIP.
int hip_fail(hipError_t e, const char* what);

constexpr int REDUCE_BLOCKS = 1024;

// A step launcher: advance one time step from `fin` to `fout` on `st`.
using StepFn = hipError_t (*)(const void* ctx, const void* fin, void* fout, hipStream_t st);

// Captured graphs of an even number of steps ping-ponging out -> scratch ->
// out, one per output buffer for the last two output buffers used (a caller
// that alternates two buffers, as a checkpointed rollout does, replays both
// without re-capturing).  The steps are captured on a stream of the
// handle's own (`cap`, created on first use), so that the graphs also serve
// callers on the null stream; a graph is then launched on the caller's
// stream, and an event recorded after its last launch lets the graph be
// destroyed only once that launch has finished.
struct StepGraph {
    struct Entry {
        hipGraphExec_t exec = nullptr;
        void* out = nullptr;
        hipEvent_t done = nullptr;   // recorded after the entry's last launch
        bool launched = false;
    };
    Entry slot[2];
    int next = 0;                    // the entry replaced next
    hipStream_t cap = nullptr;
    void drop(Entry& e);   // waits for the entry's last launch, then frees its graph
    void release();        // every graph, event and the capture stream
};


}  // namespace cdbm

struct cdbm_handle {
    cdbm_params p;
    cdbm::KParams k;
    int device = 0;
    int64_t cells = 0;
    size_t elem = 8;
    size_t fbytes = 0;
    void* scratch = nullptr;    // f-sized ping-pong buffer
    void* stage = nullptr;      // f-sized buffer of a stage-1 state (adjoint, split steps)
    bool split = false;         // step as two single-stage launches (small grids)
    bool two = false;           // two steps per launch (CDBM_STEP_FUSED2)
    void* lam_mid = nullptr;    // f-sized buffer for the adjoint's intermediate product
    double* partials = nullptr; // reduction partials
    double* tau_part = nullptr; // per-block partial sums of the adjoint's tau term (two stages)
    double* tau_acc = nullptr;  // per-block tau terms of step adjoints called without dL_dtau
    cdbm::KParams* kdev = nullptr;   // device copy of k
    int* flag = nullptr;        // device flag of the field check
    cdbm::StepGraph graph;
};

namespace cdbm {
inline bool mixed(const cdbm_handle* h) { return h->p.precision == CDBM_MIXED; }
// The compensated mixed form: float f plus the conserved-moment residual.
inline bool comp(const cdbm_handle* h) { return h->p.precision == CDBM_MIXED_COMP; }
// Planes of a state: the 16 distributions, plus the four residual planes of
// the compensated form.
inline int state_planes(int precision) { return precision == CDBM_MIXED_COMP ? NV + 4 : NV; }
int check_device(const cdbm_handle* h);
int ensure_buffer(cdbm_handle* h, void** buf);
int check_fields_range(int* flag, const double* rho, const double* ux, const double* uy,
                       const double* T, int64_t cells, hipStream_t st);

// Advance nsteps >= 1 from fin to fout (destinations alternate between fout
// and scratch and end on fout; fin is never written).  Long runs replay a
// captured graph on `st`, unless `st` is itself being captured (then every
// step is launched directly into the caller's capture).
int run_steps(StepFn fn, const void* ctx, const void* fin, void* fout, void* scratch,
              int nsteps, hipStream_t st, StepGraph& graph);
}  // namespace cdbm
