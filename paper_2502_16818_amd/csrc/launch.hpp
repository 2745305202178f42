// Host-side launchers of the CDBM kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "model.hpp"

namespace cdbm {

template <typename S>
hipError_t launch_init(const double* rho, const double* ux, const double* uy, const double* T,
                       void* f, const KParams& K, hipStream_t st);
hipError_t launch_check_fields(const double* rho, const double* ux, const double* uy,
                               const double* T, int64_t cells, int* bad, hipStream_t st);
template <typename S>
hipError_t launch_moments(const void* f, double* rho, double* ux, double* uy, double* T,
                          const KParams& K, hipStream_t st);
template <typename S>
hipError_t launch_tne(const void* f, double* out12, bool raw, const KParams& K, hipStream_t st);
template <typename S>
hipError_t launch_totals(const void* f, double* partials, int nblocks, double* out4,
                         const KParams& K, hipStream_t st);
hipError_t launch_sum_partials(const double* part, int nblocks, int ncomp, double* out,
                               hipStream_t st);
template <typename S>
hipError_t launch_stage(const void* fin, const void* base, void* fout, bool stage2,
                        const KParams& K, const KParams* Kd, hipStream_t st);

// The compensated mixed form (CDBM_MIXED_COMP): float states of 20 planes,
// the 16 of f and the four of the conserved-moment residual r.
hipError_t launch_init_comp(const double* rho, const double* ux, const double* uy,
                            const double* T, void* f, const KParams& K, hipStream_t st);
hipError_t launch_moments_comp(const void* f, double* rho, double* ux, double* uy, double* T,
                               const KParams& K, hipStream_t st);
hipError_t launch_tne_comp(const void* f, double* out12, bool raw, const KParams& K,
                           hipStream_t st);
hipError_t launch_totals_comp(const void* f, double* partials, int nblocks, double* out4,
                              const KParams& K, hipStream_t st);
hipError_t launch_stage_comp(const void* fin, const void* base, void* fout, bool stage2,
                             const KParams& K, const KParams* Kd, hipStream_t st);

// Compute units of the current device (cached per device; 256 if the query
// fails).
int device_cus();

// Fused two-stage step (kernels_step.hip).  K: host copy (launch geometry);
// Kd: the same constants in device memory (read by the kernel).
template <typename S>
hipError_t launch_step_fused(const void* fin, void* fout, const KParams& K, const KParams* Kd,
                             hipStream_t st);

// Two fused steps in one launch, FP32 storage (kernels_step.hip, step_two.hpp).
hipError_t launch_step2_fused(const void* fin, void* fout, const KParams& K, const KParams* Kd,
                              hipStream_t st);

// Adjoint (kernels_adjoint.hip).  tau_part: one double per block
// (stage_adjoint_blocks), the block sums of the launch's tau term, written
// or (tau_add) added to what it holds.
int stage_adjoint_blocks(const KParams& K);
template <typename S>
hipError_t launch_stage_adjoint(const void* f, const void* lam, const void* lam_add, void* out,
                                double* tau_part, bool tau_add, double w_in, double w_add,
                                const KParams& K, hipStream_t st);
template <typename S>
hipError_t launch_init_adjoint(const double* rho, const double* ux, const double* uy,
                               const double* T, const void* lam, double* g_rho, double* g_ux,
                               double* g_uy, double* g_T, const KParams& K, hipStream_t st);
template <typename S>
hipError_t launch_moments_adjoint(const void* f, const double* g_rho, const double* g_ux,
                                  const double* g_uy, const double* g_T, void* lam,
                                  const KParams& K, hipStream_t st);
// dst[0] += scale * sum of part[0 .. n), in a fixed order; with clear,
// part is set to zero as it is read.  Above ACCUMULATE_ONE_PASS partials a
// first pass writes ACCUMULATE_BLOCKS second-level sums into scratch
// (unused otherwise).
constexpr int ACCUMULATE_ONE_PASS = 8192, ACCUMULATE_BLOCKS = 256;
hipError_t launch_accumulate_scalar(double* part, int n, double* scratch, double scale,
                                    double* dst, bool clear, hipStream_t st);

// Batched ensemble (kernels_batch.hip).  Ks: per-grid constants (device);
// f_off: element offset of each grid's f block (device); work_start: prefix
// sums of the grids' weighted strip counts, strips * (ny + fill),
// ngrids + 1 entries (device).
template <typename S>
int batch_blocks();
// Positions a strip of the contiguous batch split weighs beyond its rows by
// default: the pipeline fill of a segment, in rows.
constexpr int BATCH_FILL = 14;
// Output columns per strip of the fused step for a precision form.
int strip_width(int precision);
// chunked: every grid's width and element offset is a multiple of the
// 16-byte chunk (the buffers' alignment is checked at launch).
template <typename S>
hipError_t launch_batch_step(const void* fin, void* fout, const KParams* Ks, const int64_t* f_off,
                             const int64_t* work_start, int ngrids, int fill, int nblocks,
                             bool chunked, hipStream_t st);

// Row-piece form of the batched step: units (device, 16-byte aligned): four
// ints per work unit, (grid, first column of its strip, first row, end
// row), in queue order; range_start (nq + 1, device): the unit ranges of
// the nq counters; counters (nq + 1 ints, device, zero before the first
// launch; the kernel leaves them zero).
template <typename S>
hipError_t launch_batch_step_rows(const void* fin, void* fout, const KParams* Ks,
                                  const int64_t* f_off, const int* units,
                                  const int64_t* range_start, int nq, int* counters, int nblocks,
                                  bool chunked, hipStream_t st);

}  // namespace cdbm
