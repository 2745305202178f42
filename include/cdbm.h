/*
 * cdbm.h - C ABI of the MI355X (gfx950) implementation of the central-moment
 * discrete Boltzmann method (CDBM) for compressible flows with a variable
 * specific-heat ratio (C. Lin, X. Su, L. Fei, K. H. Luo, arXiv:2502.16818).
 *
 * One time step, per cell and per discrete velocity i = 1..16:
 *   - macroscopic rho, u, T from the first three kinetic moments (Sec. 2,
 *     the statement after Eq. (7));
 *   - the equilibrium f_i^eq that reproduces the seven central moments of
 *     the Maxwellian, Eqs. (4)-(7) (computed as the raw-moment vector of the
 *     Maxwellian contracted with one shared inverse moment matrix; the
 *     central-to-raw shift is exact, so the result equals Eq. (7));
 *   - BGK relaxation -(f_i - f_i^eq)/tau of Eq. (1);
 *   - the NND flux-split upwind derivative with minmod, Eqs. (12)-(20);
 *   - a two-stage second-order Runge-Kutta step (Heun form).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Distributions are structure-of-arrays f[i][y][x], x fastest, i = 0..15
 *   for the paper's i = 1..16, ordered as: v_a(1,0), v_a(0,1), v_a(-1,0),
 *   v_a(0,-1); v_b(1,1), v_b(-1,1), v_b(-1,-1), v_b(1,-1); then groups c
 *   (axis) and d (diagonal) in the same order (Eq. (2)); eta_i per group
 *   (Eq. (3)).  Element type: double for CDBM_FP64, float for CDBM_MIXED.
 *   A state of CDBM_MIXED_COMP is float [20][ny][nx]: the 16 planes of f,
 *   then four planes r = (r_rho, r_jx, r_jy, r_2E) that carry what FP32
 *   storage rounded off the cell's conserved moments (see `precision`);
 *   every "[16][ny][nx]" of a state below reads "[20][ny][nx]" for it.
 * - Macroscopic fields are double arrays [y][x].
 * - Every pointer argument named as device memory must point to memory of
 *   the GPU that is current when the call is made.  The caller owns all
 *   device buffers; the library owns only its handle, a few constant and
 *   scratch buffers it allocates at creation, and captured graphs.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Calls are asynchronous on that stream unless documented otherwise.
 * - Every call returns 0 (CDBM_OK) or a negative error code; it never
 *   throws or aborts.  cdbm_last_error() returns a thread-local message
 *   describing the last failure of the calling thread.
 * - Calls on one handle must not run concurrently from several threads.
 */
#ifndef CDBM_H
#define CDBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CDBM_OK = 0,
    CDBM_EINVAL = -1,     /* an argument is out of range or inconsistent          */
    CDBM_ESINGULAR = -2,  /* the moment matrix of the velocity set is singular or
                             too ill-conditioned (block condition number > 1e10) */
    CDBM_ENONPHYS = -3,   /* rho <= 0, T <= 0 or a non-finite value in the fields */
    CDBM_EHIP = -4,       /* a HIP runtime call failed                            */
    CDBM_ENOMEM = -5      /* a library allocation failed                          */
};

enum { CDBM_PERIODIC = 0, CDBM_ZERO_GRADIENT = 1 };
enum { CDBM_FP64 = 0, CDBM_MIXED = 1, CDBM_MIXED_COMP = 2 };
enum { CDBM_STEP_AUTO = 0, CDBM_STEP_FUSED = 1, CDBM_STEP_SPLIT = 2, CDBM_STEP_FUSED2 = 3 };

/* Run parameters (Secs. 2 and 3).
 *   nx, ny      grid cells (ny = 1 for a tube); 1 <= nx, ny <= 65536 and
 *               nx*ny <= 2^28.
 *   dx, dy      cell sizes (> 0).  dt: time step (> 0).  tau: relaxation
 *               time of Eq. (1) (> 0); dt/tau <= 2 is required (the stable
 *               interval of the two-stage scheme for pure relaxation).
 *   gamma       specific-heat ratio, 1 < gamma <= 2; the extra degrees of
 *               freedom are I = 2/(gamma-1) - 2 (gamma = (D+I+2)/(D+I), D = 2,
 *               the relation stated under Eq. (5)).  Read only when
 *               dof_given = 0.
 *   v[4]        (v_a, v_b, v_c, v_d) of Eq. (2), each > 0.  Diagonal groups
 *               have components +-v (speed sqrt(2) v).
 *   eta[4]      (eta_a, eta_b, eta_c, eta_d) of Eq. (3), each >= 0.
 *   bc_x, bc_y  CDBM_PERIODIC or CDBM_ZERO_GRADIENT (two ghost layers per
 *               side copied from the edge cell before each stage).
 *   precision   CDBM_FP64: f stored and advected in double.  CDBM_MIXED: f
 *               stored and advected in float; moments, equilibrium and the
 *               relaxation difference f - f^eq in double.
 *               CDBM_MIXED_COMP: f stored in float as in CDBM_MIXED, each
 *               stage's arithmetic in double as in CDBM_FP64, and a
 *               compensation of the conserved moments: each cell also
 *               stores, in float, the part r of its mass, momentum and
 *               energy that rounding f to float removed; the cell's
 *               conserved moments are
 *               sum_i f_i psi_i + r (psi = 1, v_x, v_y, |v|^2 + eta^2), in
 *               the equilibrium, in cdbm_moments and in the totals.  A stage
 *               forms each new f_i in double, rounds it to float, and adds
 *               the conserved moments of what was rounded off to r; the
 *               relaxation towards f^eq of those moments moves r back into
 *               f (by dt/tau of it per stage).  Changes of the conserved
 *               moments far below an FP32 unit of f per step (the viscous
 *               decay of a nearly steady flow) accumulate instead of
 *               rounding away.  Runs as two single-stage launches (step_form
 *               CDBM_STEP_AUTO or CDBM_STEP_SPLIT); 20 floats per cell.  The
 *               adjoint, keep-stage and batch entry points reject it
 *               (EINVAL).
 *   step_form   how cdbm_step runs a time step; all forms give the same
 *               result up to rounding order.  CDBM_STEP_FUSED: both stages
 *               in one launch that streams strips of the grid through LDS
 *               (f crosses HBM once in and once out per step).
 *               CDBM_STEP_SPLIT: two single-stage launches, one cell per
 *               thread, f^(1) through a handle-owned buffer (faster on small
 *               grids, where the fused launch has too few strips to fill the
 *               chip).  CDBM_STEP_AUTO: split up to 2^19 cells (724 x 724)
 *               in the mixed form and 2^18 (512 x 512) in FP64, fused
 *               above.  CDBM_STEP_FUSED2 (CDBM_MIXED only): two time steps
 *               per launch (temporal blocking: f crosses HBM once in and
 *               once out per two steps, on 48-column strips that carry four
 *               rings of stages in LDS); an odd last step runs fused.  Same
 *               results as CDBM_STEP_FUSED bit for bit.  Ignored by the
 *               batched form (always fused).
 *   dof_given   0: the gas is given by gamma.  1: it is given by the extra
 *               degrees of freedom `extra_dof` = I >= 0 of Eq. (5) (finite),
 *               and gamma is ignored.  A zero-initialised struct selects
 *               gamma. */
typedef struct cdbm_params {
    int32_t nx, ny;
    double dx, dy, dt, tau;
    double gamma;
    double v[4];
    double eta[4];
    int32_t bc_x, bc_y;
    int32_t precision;
    int32_t step_form;
    int32_t dof_given;
    double extra_dof;
} cdbm_params;

typedef struct cdbm_handle cdbm_handle;
typedef struct cdbm_batch cdbm_batch;

/* Thread-local description of the calling thread's last error ("" if none). */
const char* cdbm_last_error(void);

/* Validate `p`, build the 16x16 moment matrix of the velocity set at u = 0
 * (rows of Eq. (6)), split it into its four parity blocks and invert them in
 * extended precision on the host; allocate the handle's scratch (one f-sized
 * ping-pong buffer and reduction partials) on the current device.
 * Synchronous.  Errors: EINVAL, ESINGULAR, ENOMEM, EHIP.
 *
 * Setting up a run is two calls: cdbm_create (parameters, constants and
 * allocations; synchronous, no fields) and cdbm_init (f = f^eq of the
 * initial fields into a caller buffer; asynchronous after its field check).
 * An initialiser that takes the parameters and the fields and returns a
 * handle is exactly cdbm_create followed by cdbm_init; keeping them apart
 * lets one handle initialise many states (ensembles, the target runs of a
 * gradient problem) without rebuilding the constants. */
int cdbm_create(const cdbm_params* p, cdbm_handle** out);

/* Release everything the handle owns.  NULL is accepted.  Synchronizes the
 * device before freeing. */
int cdbm_destroy(cdbm_handle* h);

/* Copy of the parameters the handle was created with. */
int cdbm_get_params(const cdbm_handle* h, cdbm_params* out);

/* f = f^eq(rho, u, T) in every cell (the initial condition used in Sec. 3).
 * rho, ux, uy, T: device double [ny][nx]; f_out: device [16][ny][nx].
 * Checks the fields on the device first and returns ENONPHYS (f_out
 * untouched) if any rho or T is <= 0 or any value is not finite; this check
 * synchronizes `stream`. */
int cdbm_init(cdbm_handle* h, const double* rho, const double* ux, const double* uy,
              const double* T, void* f_out, void* stream);

/* Advance `nsteps` >= 0 time steps of Eq. (1) (NND in space, Eqs. (12)-(20);
 * Heun RK2 in time) from f_in to f_out (device [16][ny][nx]).  f_in is not
 * modified; f_out must not overlap f_in.  The library ping-pongs between
 * f_out and its own scratch buffer so that the result lands in f_out.
 * nsteps = 0 copies f_in to f_out. */
int cdbm_step(cdbm_handle* h, const void* f_in, void* f_out, int32_t nsteps, void* stream);

/* Macroscopic fields of f (Sec. 2, statement after Eq. (7)): rho = sum f_i,
 * rho u = sum f_i v_i, rho (D+I) T = sum f_i (|v_i - u|^2 + eta_i^2).
 * Outputs: device double [ny][nx] each. */
int cdbm_moments(cdbm_handle* h, const void* f, double* rho, double* ux, double* uy,
                 double* T, void* stream);

/* Thermodynamic nonequilibrium measures, Eqs. (8)-(11):
 * out12[k][y][x] (device double, 12 planes) = sum_i (f_i - f_i^eq) Psi_{k+5}(v_i - u)
 * in the row order of Eq. (6): Delta*_2 (xx, xy, yy), Delta*_{3,1} (x, y),
 * Delta*_3 (xxx, xxy, xyy, yyy), Delta*_{4,2} (xx, xy, yy). */
int cdbm_tne(cdbm_handle* h, const void* f, double* out12, void* stream);

/* The same twelve measures in the raw-moment construction that Sec. 2
 * contrasts the CDBM with: sum_i (f_i - f_i^eq) Psi_{k+5}(v_i) at the raw
 * velocities v_i instead of the peculiar ones v_i - u, same f^eq (the raw
 * and central moment constraints of Eqs. (4)-(7) have the same solution for
 * this set of sixteen moment functions) and the same slot order as cdbm_tne.
 * Delta_2 = Delta*_2 (the mass and momentum of f - f^eq vanish), while the
 * higher measures pick up the flow: Delta_{3,1} = Delta*_{3,1} + 2 Delta*_2 u,
 * and so on.  out12: device double,
 * 12 planes of [ny][nx]. */
int cdbm_tne_raw(cdbm_handle* h, const void* f, double* out12, void* stream);

/* Grid totals of mass, x- and y-momentum and energy (sum over cells of
 * rho, rho u_x, rho u_y and sum_i f_i (|v_i|^2 + eta_i^2)), accumulated in
 * double.  out4: device double[4], overwritten. */
int cdbm_conserved_totals(cdbm_handle* h, const void* f, double* out4, void* stream);

/* cdbm_conserved_totals for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): no handle, no hipMalloc or hipFree.  p: the parameters of the
 * grid f belongs to (validated as by cdbm_create; only nx, ny, v, eta and
 * precision affect the result); f, out4: as for cdbm_conserved_totals, whose
 * result this equals bit for bit.  The block partial sums live in a 32 KiB
 * array allocated statically in the library on each GPU and held until the
 * process ends; its size does not depend on the grid, so every grid the
 * parameters allow fits.  Every call on a GPU uses that GPU's one array:
 * calls that overlap in time on one GPU (other streams, other threads)
 * race and give wrong totals; order them on one stream.  The first call on
 * each GPU looks up the array's device address (synchronous, not a stream
 * operation); make it outside a graph capture. */
int cdbm_conserved_totals_static(const cdbm_params* p, const void* f, double* out4, void* stream);

/* Reverse-mode product of one time step F (the map of cdbm_step with
 * nsteps = 1): lam_n = (dF/df)^T(f_n) lam_np1 and *dL_dtau += (dF/dtau)^T lam_np1.
 * f_n: device [16][ny][nx] in the handle's precision.  lam_np1, lam_n:
 * device double [16][ny][nx] in both precision forms (adjoint vectors carry
 * gradients in small deviations between velocities that FP32 would round
 * away); lam_n must not overlap f_n or lam_np1.  dL_dtau: device double[1],
 * accumulated (never overwritten); or NULL, and the step's dL/dtau term is
 * added to the handle's accumulator instead, one double per block of the
 * stage-adjoint launch, to be summed by cdbm_tau_collect (a reverse pass
 * over many steps then pays for one sum instead of one per step; the total
 * differs from per-step sums by rounding order only).  minmod passes the
 * derivative to its first argument on a tie |X| = |Y| and none when its
 * value is 0 (the branch order of Eq. (16)).  Uses the handle's scratch
 * buffer, so calls on one handle must be ordered on one stream. */
int cdbm_step_adjoint(cdbm_handle* h, const void* f_n, const void* lam_np1, void* lam_n,
                      double* dL_dtau, void* stream);

/* One time step (cdbm_step with nsteps = 1) that also keeps its first
 * Runge-Kutta stage (Sec. 2: the second-order Runge-Kutta scheme in time;
 * with Eq. (1) and the NND derivative of Eqs. (12)-(20) as L):
 * f1_out = f_in + dt L(f_in) and f_out = f_in / 2 + (f1_out + dt L(f1_out)) / 2,
 * as two single-stage launches whatever the handle's step form.  f_in, f1_out,
 * f_out: device [16][ny][nx] in the handle's precision, pairwise
 * non-overlapping.  f_out equals what cdbm_step gives for one step bit for
 * bit.  Meant for reverse passes that keep the stages of recomputed steps
 * (see cdbm_step_adjoint_stage).  It writes no buffer of the handle, so it
 * may run on another stream at the same time as the handle's step adjoints
 * (on buffers they do not read). */
int cdbm_step_keep_stage(cdbm_handle* h, const void* f_in, void* f1_out, void* f_out,
                         void* stream);

/* cdbm_step_adjoint with the first Runge-Kutta stage of the step supplied
 * instead of recomputed: f1 = f_n + dt L(f_n) (device [16][ny][nx], handle's
 * precision), as cdbm_step_keep_stage writes it.  Same arguments, contract
 * and results as cdbm_step_adjoint (bit for bit when f1 is that stage);
 * lam_n must not overlap f1 either.  Saves one single-stage launch. */
int cdbm_step_adjoint_stage(cdbm_handle* h, const void* f_n, const void* f1,
                            const void* lam_np1, void* lam_n, double* dL_dtau, void* stream);

/* *dL_dtau += the sum, in a fixed order, of the dL/dtau terms that step
 * adjoints called with dL_dtau = NULL have added to the handle's accumulator
 * since the handle was created or last collected; the accumulator is
 * cleared (no step adjoint with NULL may run in between on another stream).
 * dL_dtau: device double[1].  Two launches at most, no allocation. */
int cdbm_tau_collect(cdbm_handle* h, double* dL_dtau, void* stream);

/* Reverse-mode product of cdbm_init: g_q = (d f^eq(q) / d q)^T lam_f0 for
 * q = (rho, u_x, u_y, T) taken from the given fields (device double [ny][nx]).
 * lam_f0: device double [16][ny][nx].  Outputs overwritten. */
int cdbm_init_adjoint(cdbm_handle* h, const double* rho, const double* ux, const double* uy,
                      const double* T, const void* lam_f0, double* g_rho, double* g_ux,
                      double* g_uy, double* g_T, void* stream);

/* Reverse-mode product of cdbm_moments: lam_f = (d(rho, u, T)/df)^T g.
 * f: device [16][ny][nx] in the handle's precision; g_*: device double
 * [ny][nx]; lam_f: device double [16][ny][nx], overwritten. */
int cdbm_moments_adjoint(cdbm_handle* h, const void* f, const double* g_rho,
                         const double* g_ux, const double* g_uy, const double* g_T,
                         void* lam_f, void* stream);

/* Batched ensemble of independent grids advanced by one launch per step.
 * per_grid[k]: parameters of grid k; v, eta and precision must be the same
 * for all grids (one shared inverse moment matrix), everything else may
 * differ.  f_offsets[k]: element offset of grid k's [16][ny][nx] block inside
 * the caller's batch buffers (blocks must not overlap).  Both arrays are
 * host memory, copied.  Synchronous.  Errors as cdbm_create. */
int cdbm_batch_create(const cdbm_params* per_grid, int32_t ngrids, const int64_t* f_offsets,
                      cdbm_batch** out);
int cdbm_batch_destroy(cdbm_batch* b);

/* f = f^eq of the fields of every grid.  The four fields are concatenated
 * grid after grid (grid k's cells start at f_offsets[k] / 16).
 * Same checks and synchronization as cdbm_init. */
int cdbm_batch_init(cdbm_batch* b, const double* rho, const double* ux, const double* uy,
                    const double* T, void* f_out, void* stream);

/* Advance every grid of the batch by nsteps (each with its own dt, tau,
 * gamma, dx, dy, sizes and boundary conditions).  Same buffer contract as
 * cdbm_step; the per-step launch is captured once into a HIP graph and
 * replayed. */
int cdbm_batch_step(cdbm_batch* b, const void* f_in, void* f_out, int32_t nsteps, void* stream);

/* How the batched step spreads the grids' strips over its persistent
 * blocks (one block per compute unit); every layout gives bit-identical
 * results.
 *   CDBM_BATCH_CONTIGUOUS: the (grid, strip, row) sequence cut into equal
 *     contiguous pieces, one per block, each strip weighing its rows plus
 *     fill_rows (the pipeline fill of a segment; default 14).
 *   CDBM_BATCH_ROW_PIECES: every grid cut into row pieces of about
 *     piece_rows rows; the units (grid, piece, strip) are taken in order from
 *     one counter per XCD, so that the blocks of an XCD work on neighbouring
 *     strips of the same rows at the same time, and a block whose XCD's
 *     units are used up takes units from the other XCDs' counters.  With
 *     tail_rows > 0 the last tail_rows rows of every grid taller than twice
 *     that are cut off the pieces and taken, one unit per strip, after the
 *     pieces of the same counter, so that each counter ends with small
 *     units.
 * tail_rows must be 0 in the contiguous layout. */
enum { CDBM_BATCH_CONTIGUOUS = 0, CDBM_BATCH_ROW_PIECES = 1 };
typedef struct cdbm_batch_launch {
    int32_t layout;
    int32_t fill_rows;    /* CONTIGUOUS: 0 .. 1024 */
    int32_t piece_rows;   /* ROW_PIECES: 16 .. 65536 */
    int32_t tail_rows;    /* ROW_PIECES: 0, or 8 .. 65536 */
} cdbm_batch_launch;

/* The batch's current launch layout. */
int cdbm_batch_get_launch(const cdbm_batch* b, cdbm_batch_launch* out);

/* Select a launch layout (synchronous: uploads its tables; drops the
 * captured step graphs).  Errors: EINVAL for a layout out of range. */
int cdbm_batch_set_launch(cdbm_batch* b, const cdbm_batch_launch* l);

/* Autotuner of the batched step.  Looks up the batch's key (the device's gfx
 * architecture, the precision form, and floor(log2) of the batch's cell and
 * grid counts) in the JSON cache file `cache_path` (NULL: no cache) and
 * applies the stored layout; otherwise times the candidate layouts (the
 * contiguous split with fill_rows 0, 14, 28; row pieces of 128 and 192
 * rows; row pieces with tails, (piece_rows, tail_rows) = (160, 64),
 * (192, 64), (320, 96), (320, 128), (384, 160), (448, 160); 26 steps each),
 * applies the fastest and adds it to the cache
 * (written through a temporary file; an unwritable cache is skipped).  f_in:
 * a state of the batch (read only); f_out and the batch's scratch buffer are
 * overwritten by the timing steps.  `chosen` (may be NULL) receives the
 * layout applied.  Synchronous. */
int cdbm_batch_autotune(cdbm_batch* b, const void* f_in, void* f_out, const char* cache_path,
                        cdbm_batch_launch* chosen, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CDBM_H */
