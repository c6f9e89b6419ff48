/*
 * wavestep.h -- C ABI of the MI355X (gfx950) time step of the hybrid
 * finite-volume / finite-difference extended-Boussinesq solver of
 * Tavakkol & Lynett, "Celeris" (arXiv:1611.05984).
 *
 * One time step (sec. 2.3) = a predictor pass (third-order Adams-Bashforth,
 * eqs. 15-17) and n_corr corrector passes (fourth-order Adams-Moulton,
 * eqs. 18-20).  Each pass evaluates the right-hand side (KP07 central-upwind
 * fluxes with generalized-minmod reconstruction, positivity correction and
 * desingularized velocities, sec. 2.2 steps 1-4 and eq. 14; central
 * finite-difference dispersive terms of eqs. 10-13; friction eqs. 31-32),
 * integrates w, U*, V*, and recovers P and Q from the row and column
 * tridiagonal systems of eqs. 21-23.  Boundaries: solid walls (sec. 2.4.1),
 * sine/irregular wave makers (sec. 2.4.2, eqs. 25-29), sponge layers
 * (sec. 2.4.3, eq. 30).  Solitary waves: sec. 2.7, eqs. 33-36.
 *
 * Conventions
 *  - Every length is in metres, every time in seconds, g in m/s^2.
 *  - Cells (i, j), i in [0, nx), j in [0, ny), centre ((i+1/2)dx, (j+1/2)dy).
 *    2-D arrays are row-major with x fastest; "pitch" is the row stride in
 *    elements (>= nx).
 *  - Bathymetry is the bottom elevation z at the cell corners (i dx, j dy),
 *    (ny+1) rows of (nx+1) values, above the same datum as the water surface
 *    w; the bottom is continuous and bilinear between corners.
 *  - Device pointers are HIP device addresses; "stream" is a hipStream_t
 *    (NULL = the null stream).  Calls that take a stream are asynchronous
 *    unless stated otherwise.
 *  - Ownership: the caller allocates the workspace (ws_workspace_bytes()) and
 *    every array it passes; the library borrows the workspace until
 *    ws_domain_destroy() and never frees caller memory.  Host arrays are read
 *    only during the call.  Handles are library-owned; one handle must not be
 *    used from two threads at once.
 *  - Errors: every call returns a ws_status; nothing aborts or throws across
 *    the ABI.  ws_last_error() returns a thread-local description of the last
 *    failure.  Faults found by kernels (non-finite state) set a per-domain
 *    health word that the next synchronous call (ws_query) reports.
 */
#ifndef WAVESTEP_H
#define WAVESTEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ws_domain ws_domain; /* opaque, library-owned */
typedef struct ws_batch ws_batch;   /* opaque, library-owned */

typedef enum {
    WS_OK = 0,
    WS_EINVAL = -1,      /* bad argument                                        */
    WS_ENOMEM = -2,      /* workspace too small / host allocation failed        */
    WS_EHIP = -3,        /* a HIP runtime call failed                           */
    WS_ENOTDD = -4,      /* a row/column system of eq. 23 is not diagonally dominant */
    WS_ENONFINITE = -5,  /* the state became non-finite                         */
    WS_EBUSY = -6        /* batch full / slot in use                            */
} ws_status;

enum { WS_BSNQ = 0, WS_NLSW = 1 };                               /* model (sec. 3.2)  */
enum { WS_FRIC_NONE = 0, WS_FRIC_QUAD = 1, WS_FRIC_MANNING = 2 }; /* eqs. 31, 32       */
enum { WS_WEST = 0, WS_EAST = 1, WS_SOUTH = 2, WS_NORTH = 3 };
enum { WS_BC_SOLID = 0, WS_BC_SPONGE = 1, WS_BC_WAVES = 2 };     /* sec. 2.4          */
enum { WS_EDIT_ADD_WATER = 0, WS_EDIT_RAISE_TERRAIN = 1 };       /* sec. 1 edits      */
enum { WS_READ_W = 0, WS_READ_H = 1 };                           /* first field of ws_read */

/* Grid and model parameters.  Defaults in brackets follow the paper: B = 1/15
 * (sec. 2.1), eps = 5e-12 and two correctors (Fig. 2), g = 9.81, theta = 1.3
 * (generalized minmod, sec. 2.2 step 1; the paper gives no value).
 * fstar_extrap selects the predictor's extrapolation of F*, G*: 2 = the
 * quadratic form printed in eqs. 16-17, 1 = linear (default; the printed form
 * is linearly unstable in 2-D with two correctors once d/dx > ~4.5), 0 = none.
 * The first two steps after ws_domain_init / ws_set_state are first-order
 * Euler steps without correctors (sec. 2.3). */
typedef struct {
    int32_t nx, ny;          /* cells, >= 2 each; five padded fields (nx rounded  */
                             /* up to 64, ny to 16, 4 B a cell) must stay under   */
                             /* 4 GiB: about 2.1e8 cells (squares up to 14640^2)  */
    int32_t n_corr;          /* corrector passes per step [2]                     */
    int32_t model;           /* WS_BSNQ or WS_NLSW [WS_BSNQ]                      */
    int32_t friction;        /* WS_FRIC_* [WS_FRIC_NONE]                          */
    int32_t fstar_extrap;    /* 0, 1 or 2 [1]                                     */
    double dx, dy, dt;       /* spacing and fixed time step, > 0                  */
    double g;                /* [9.81]                                            */
    double still_water;      /* still water surface elevation w_s [0]             */
    double Bcoef;            /* dispersion coefficient B [1/15]                   */
    double theta;            /* minmod parameter in [1, 2] [1.3]                  */
    double eps;              /* desingularization tolerance of eq. 14 [5e-12]     */
    double friction_coef;    /* f of eq. 31 or Manning n of eq. 32 [0]            */
} ws_grid;

/* One side's boundary condition.  WS_BC_WAVES superposes n_comp sine
 * components (eqs. 25-28; wave number from Eckart's eq. 29 at ref_depth, or,
 * when ref_depth <= 0, at the mean still water depth of the first interior
 * row/column along that side).  WS_BC_SPONGE is a wall whose width_cells
 * nearest cells are damped once per step by eq. 30.  Host arrays, length
 * n_comp (<= 256), read during the call; phase may be NULL (zeros). */
typedef struct {
    int32_t type;            /* WS_BC_*                                           */
    int32_t width_cells;     /* sponge width in cells                             */
    int32_t n_comp;          /* wave components                                   */
    int32_t reserved;
    const double *amp;       /* amplitude a, m                                    */
    const double *period;    /* period T, s                                       */
    const double *theta_rad; /* direction from +x, radians                        */
    const double *phase;     /* phase offset, radians                             */
    double ref_depth;        /* m; <= 0: mean depth along the side                */
    double sponge_reflect;   /* WS_BC_SPONGE: target reflection coefficient R in  *
                              * [0, 1] of long waves (0: the layer of eq. 30).    *
                              * The layer's factor becomes gamma^s with           *
                              * s = min(1, -ln(R) c dt / (4 L ln 2)): a long wave *
                              * (c = sqrt(g d), d the mean still water depth next *
                              * to the side) that crosses the layer of width L    *
                              * and comes back keeps the share R of its amplitude *
                              * (int_0^L ln gamma = -2 L ln 2).  R = 1 leaves a   *
                              * solid wall.  The paper names partially reflective *
                              * sponges without a formula; this is the reading.   */
} ws_boundary;

/* Fill *g with the defaults above for an nx x ny grid (dx, dy, dt left 0). */
void ws_grid_defaults(ws_grid *g, int32_t nx, int32_t ny);

/* Device bytes the caller must supply to ws_domain_init for this grid
 * (0 if the grid is invalid). */
size_t ws_workspace_bytes(const ws_grid *g);

/* Create a domain in the caller's device workspace.  z_corners_dev: device
 * array of (ny+1)*(nx+1) floats, bathymetry at the cell corners (copied; the
 * caller may free it after the call returns).  All sides start as solid walls
 * and the state as a lake at rest (w = max(w_s, cell bottom), P = Q = 0).
 * Synchronous.  Returns WS_ENOTDD if a system of eq. 23 is not diagonally
 * dominant (bed too steep for the grid). */
ws_status ws_domain_init(const ws_grid *g, const float *z_corners_dev, void *workspace_dev,
                         size_t workspace_bytes, void *stream, ws_domain **out);

ws_status ws_domain_destroy(ws_domain *d);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: work being captured into a graph elsewhere, tight serving loops,
 * harnesses that forbid allocation).  The same as ws_domain_init, except that
 * the workspace is the library's own static device array of
 * WS_STATIC_WORKSPACE_BYTES (80 MiB: grids up to 1024 x 512 or 768 x 768
 * cells; about 130 bytes a cell of the grid padded to whole 64 x 16 tiles,
 * as ws_workspace_bytes reports), one per GPU, held from the library's first use
 * on that GPU until the process ends, and that the handle lives in static
 * storage: the call allocates nothing, on the device or on the host.  It
 * uses the array of the device current at the call (`stream` must belong to
 * it).  The array is cleared at every such init (a destroyed domain's
 * contents do not carry over).  One such domain per device at a time:
 * WS_EBUSY while another one on the same device is alive (ws_domain_destroy
 * releases the array); WS_ENOMEM, with the sizes in ws_last_error(), if the
 * grid needs more than the array holds.  Every other call works on the
 * returned handle as on any domain.  Work on two such domains of one device
 * cannot overlap, since there is only one; two threads calling this on one
 * device race for the array, and the second gets WS_EBUSY.  Synchronous. */
#define WS_STATIC_WORKSPACE_BYTES ((size_t)80 << 20)
ws_status ws_domain_init_static(const ws_grid *g, const float *z_corners_dev, void *stream,
                                ws_domain **out);

/* Boundary condition of one side (WS_WEST..WS_NORTH).  Synchronous. */
ws_status ws_set_boundary(ws_domain *d, int32_t side, const ws_boundary *b);

/* Change parameters of a running domain (the paper's interactive changes of
 * the physical and numerical parameters, sec. 3.3): model, friction and its
 * coefficient, B, theta, eps, g, fstar_extrap and dt take effect at the next
 * step; nx, ny, dx, dy, n_corr and still_water must equal the current ones
 * (WS_EINVAL).  A new dt restarts the multistep history (the next two steps
 * are Euler steps, as after ws_set_state; the step count restarts from 0, the
 * time goes on) and rescales partially reflective sponges; a new model or B
 * refactors the reduced systems and is refused with WS_ENOTDD, the domain
 * unchanged, if eq. 23 would lose diagonal dominance (that check
 * synchronizes `stream`).  The state is kept. */
ws_status ws_update_grid(ws_domain *d, const ws_grid *g, void *stream);

/* Hot start (sec. 3.2): device arrays w (surface elevation), P, Q with row
 * pitch `pitch` elements; t is the time of this state.  Restarts the
 * multistep history (the next two steps are Euler steps). */
ws_status ws_set_state(ws_domain *d, const float *w, const float *P, const float *Q,
                       int32_t pitch, double t, void *stream);

/* Gauges (sec. 3.2: the solver can save w, P, Q at chosen grid points only).
 * ij_dev: device array of n cell index pairs (i, j); out_dev: device array of
 * 4n floats receiving (w, h = w - cell bottom, P, Q) of each gauge's cell in
 * the current state; a pair outside the grid gives four NaNs.  Asynchronous
 * and allocation-free, so a caller can record a time series by pointing
 * out_dev at successive rows of its own buffer between steps. */
ws_status ws_read_gauges(ws_domain *d, int32_t n, const int32_t *ij_dev, float *out_dev, void *stream);

/* Superpose a solitary wave of height H (sign allowed), direction theta
 * (radians), crest through (x0, y0), eqs. 33-36, where the still water depth
 * is positive.  The depth of eqs. 35-36 is the still water depth of the
 * bilinear bottom at (x0, y0); WS_EINVAL if that is not positive. */
ws_status ws_add_solitary(ws_domain *d, double H, double theta, double x0, double y0,
                          void *stream);

/* Advance nsteps full time steps (predictor + n_corr correctors each).
 * Asynchronous on `stream`. */
ws_status ws_advance(ws_domain *d, int64_t nsteps, void *stream);

/* Copy the state to device arrays (row pitch `pitch`): first field w
 * (what = WS_READ_W) or depth h = w - cell bottom (WS_READ_H), then P, Q.
 * Any pointer may be NULL.  Asynchronous. */
ws_status ws_read(ws_domain *d, int32_t what, float *first, float *P, float *Q, int32_t pitch,
                  void *stream);

/* Interactive edit (sec. 1): add a Gaussian hump amp*exp(-r^2/(2 sigma^2))
 * centred at (x0, y0) to the water surface (WS_EDIT_ADD_WATER) or to the
 * terrain corners (WS_EDIT_RAISE_TERRAIN; amp < 0 lowers it).  A terrain
 * edit keeps the free surface and scales P, Q by the cell's remaining depth
 * over its old depth (at most 1: the depth-averaged velocity is kept where
 * the cell stays wet).  The surface is then kept at or above the bottom and
 * P, Q are desingularized where the water is thinner than eps^(1/4).  A terrain edit that would make a system
 * of eq. 23 lose diagonal dominance is rejected with WS_ENOTDD and changes
 * nothing.  Synchronous for terrain edits, asynchronous for water edits. */
ws_status ws_apply_edit(ws_domain *d, int32_t kind, double x0, double y0, double amp,
                        double sigma, void *stream);

/* Snapshot / restore (checkpoint, session migration).  A snapshot holds the
 * current state, the multistep history, the (possibly edited) bathymetry,
 * the step count and the time, in a caller-owned device buffer of
 * ws_snapshot_bytes(d) bytes (256-byte aligned).  Boundary settings are not
 * part of it.  ws_snapshot is asynchronous on `stream`; ws_restore reads the
 * header synchronously, returns WS_EINVAL if the snapshot was taken from a
 * domain of another grid size, corrector count or model, then copies
 * asynchronously.  Stepping on after a restore continues the run exactly as
 * it would have continued from the snapshot.  A snapshot taken while the
 * domain ran at another time step (ws_update_grid changed dt since) restores
 * its state, bathymetry and time but restarts the multistep history: the
 * step count becomes 0 and the next two steps are Euler steps, since history
 * levels spaced by the old dt do not fit the multistep formulas at the new
 * one. */
size_t ws_snapshot_bytes(const ws_domain *d);
/* The same for a grid not yet created (0 if the grid is invalid): what a
 * caller budgeting device memory for a domain and its checkpoint needs. */
size_t ws_snapshot_bytes_grid(const ws_grid *g);
ws_status ws_snapshot(ws_domain *d, void *dst_dev, size_t bytes, void *stream);
ws_status ws_restore(ws_domain *d, const void *src_dev, size_t bytes, void *stream);

/* Synchronize `stream` and report the number of completed steps, the
 * simulated time and the health word (0 = finite state).  Returns
 * WS_ENONFINITE when the health word is set. */
ws_status ws_query(ws_domain *d, void *stream, int64_t *step, double *t, int32_t *health);

/* Kernel timing for measurement.  While enabled, ws_advance brackets every
 * kernel launch with HIP events recorded on the launch stream.
 * ws_profile_collect synchronizes `stream`, adds each kernel class's summed
 * duration (ms) and launch count into total_ms[k] / launches[k] for
 * k < n (classes WS_K_*), and clears the recorded events. */
enum { WS_K_PREDICTOR = 0, WS_K_CORRECTOR = 1, WS_K_REDUCE = 2, WS_K_SOLVE = 3, WS_K_EXPAND = 4,
       WS_K_COUNT = 5 };
ws_status ws_profile_enable(ws_domain *d, int32_t on);
ws_status ws_profile_collect(ws_domain *d, void *stream, double *total_ms, int64_t *launches,
                             int32_t n);

/* ---- Batches: many independent domains advanced together (the ensemble
 * and serving forms).  Each phase of a pass is one launch for all attached
 * domains; the per-domain step bookkeeping (Euler start-up, history slots,
 * buffer rotation) lives on the device, so a step is captured once as a HIP
 * graph on a non-null stream and replayed.  Domains of any size and at any
 * step index mix in one batch.  The caller allocates the batch workspace
 * (ws_batch_workspace_bytes) and keeps every attached domain alive.
 * While attached, a domain is advanced only by ws_batch_advance; after it,
 * ws_batch_sync must run before any per-domain call on an attached domain
 * (they return WS_EBUSY until then).  Edits, hot starts and boundary changes
 * on an attached, synced domain are allowed and picked up by the next
 * ws_batch_advance. */
size_t ws_batch_workspace_bytes(int32_t max_domains);
ws_status ws_batch_create(int32_t max_domains, void *workspace_dev, size_t workspace_bytes,
                          ws_batch **out);
ws_status ws_batch_destroy(ws_batch *b);
/* Attach a domain (WS_EBUSY if the batch is full or the domain attached
 * elsewhere).  No device call: may run while the batch's steps are in
 * flight; the domain joins at the next ws_batch_advance. */
ws_status ws_batch_attach(ws_batch *b, ws_domain *d, int32_t *slot);
ws_status ws_batch_detach(ws_batch *b, int32_t slot);
/* Step limit of one attached domain: the batch does not advance it past
 * step `stop_step` (completed steps, as ws_query reports; -1 = no limit), so
 * sessions pause at their next edit while the rest of the batch runs on.
 * Takes effect at the next ws_batch_advance; no device call. */
ws_status ws_batch_set_stop(ws_batch *b, int32_t slot, int64_t stop_step);
/* Advance every attached domain by nsteps full steps (fewer for a domain
 * that reaches its step limit).  Asynchronous. */
ws_status ws_batch_advance(ws_batch *b, int64_t nsteps, void *stream);
/* Synchronize `stream` and bring the attached domains' step, time and state
 * buffer index up to date on the host. */
ws_status ws_batch_sync(ws_batch *b, void *stream);
/* Step, simulated time and health word (0 = finite) of the domain in `slot`
 * as of the last ws_batch_sync; host only, no device call.  WS_EBUSY if the
 * batch has advanced since. */
ws_status ws_batch_status(ws_batch *b, int32_t slot, int64_t *step, double *t, int32_t *health);

/* ---- Corrector iteration until convergence (sec. 2.3: the corrector is
 * iterated a set number of times or until the variables converge).
 * With tol_w > 0, every full step of ws_advance iterates the corrector until
 * the largest change over the interior cells between two successive
 * iterates (the predictor's being the first) is at most tol_w for w (m) and
 * at most tol_pq for P and Q (m^2/s), or until n_corr correctors have run
 * (the grid's n_corr is the cap; the Euler start-up steps run none).  The
 * sponge follows the last corrector as always.  Each test is a device
 * reduction and an 8-byte read-back, so ws_advance synchronizes its stream
 * once per corrector in this mode.  tol_w <= 0 restores the fixed count (the
 * default).  Resets the counters of ws_corrector_stats.  WS_EBUSY for a
 * domain attached to a batch; ws_batch_attach refuses (WS_EINVAL) a domain
 * in this mode. */
ws_status ws_set_corrector_tolerance(ws_domain *d, double tol_w, double tol_pq);
/* Correctors the last step ran and the total since the tolerance was set;
 * the changes of w and of P, Q measured after the last corrector (tolerance
 * mode only; any pointer may be NULL).  Host only. */
ws_status ws_corrector_stats(const ws_domain *d, int32_t *last, int64_t *total, double *dw, double *dpq);

/* ---- Tuning: launch shapes chosen per grid shape.
 * stencil_rows: rows each stencil workgroup streams (8, 16, 24, 32, 48 or
 * 64; taller strips repeat fewer warm-up rows, shorter ones give more
 * workgroups and a smaller last wave of workgroups) in the predictor pass,
 * and in the corrector passes too unless corrector_rows (same choices) is
 * set: the predictor moves twice the corrector's bytes and the corrector
 * is bound by instruction issue, so their best heights can differ; 0 =
 * stencil_rows for every pass.  pcr_threads: threads
 * per reduced tridiagonal system in the partitioned solve (64, 128 or 256:
 * equations held per thread versus threads per barrier).  solver: the
 * reduced systems by PCR (WS_SOLVE_PCR) or by the Thomas algorithm with one
 * lane per system (WS_SOLVE_THOMAS: linear work, no barriers, a dependent
 * chain per lane) or by factors computed once per bathymetry and boundary
 * set (WS_SOLVE_LU: the same Thomas arithmetic, two multiply-adds per unknown
 * per pass, system-interleaved storage; systems of up to 512 unknowns, i.e.
 * grids up to 4096 cells in a direction, run as one workgroup per 64
 * systems with the systems in registers, longer ones lane per system;
 * refactored automatically after ws_set_boundary, terrain edits and
 * ws_restore) or by such factors of a
 * two-ended elimination (WS_SOLVE_LU2: two lanes per system meeting in the
 * middle, half the dependent chain) or by PCR on a single wave per system
 * (WS_SOLVE_PCR_WAVE: each lane holds equations k = lane + 64 j; the levels
 * of stride below 64 exchange equations by lane shuffles, the longer ones
 * within a lane's registers; no LDS array and no barrier; reduced systems of
 * up to 512 unknowns, i.e. grids up to 4096 cells in a direction:
 * ws_set_tuning returns WS_EINVAL for longer ones, and a batch whose largest
 * system is longer runs the workgroup PCR instead, which gives the same
 * bits).  The autotuners time each strategy together with the reduction it
 * needs (the factored solves' reduction writes right-hand sides only).
 * Rows and threads do not change results (bitwise); THOMAS and LU give
 * the same bits, and so do PCR and PCR_WAVE; PCR, LU and LU2 round the
 * reduced solve differently. */
enum { WS_SOLVE_PCR = 0, WS_SOLVE_THOMAS = 1, WS_SOLVE_LU = 2, WS_SOLVE_LU2 = 3,  /* reduced-system strategy */
       WS_SOLVE_PCR_WAVE = 4 };
typedef struct {
    int32_t stencil_rows;
    int32_t pcr_threads;
    int32_t solver;
    int32_t corrector_rows;
    int32_t reserved[4];
} ws_tuning;
ws_status ws_get_tuning(const ws_domain *d, ws_tuning *out);
ws_status ws_set_tuning(ws_domain *d, const ws_tuning *t);
/* Tuning of a batch (shared by its domains; default 32 rows, 128 threads). */
ws_status ws_batch_set_tuning(ws_batch *b, const ws_tuning *t);
/* Autotuner: times every candidate launch shape on this domain's grid
 * (predictor- and corrector-pass stencils and the reduced solves, HIP events
 * on `stream`; the state, the step and the history levels the next step
 * reads are not changed, so results are unaffected), applies the fastest and
 * returns it in *out.  With a cache file (may be NULL), a shape already
 * measured is read from it instead, and new results are appended to it as
 * lines "nx ny n_corr model stencil_rows pcr_threads solver corrector_rows"
 * (lines without the last field are read with corrector_rows = 0).
 * Timing a predictor pass rewrites the history level and corrector bases
 * the next step's predictor rewrites anyway.  Synchronous. */
ws_status ws_tune(ws_domain *d, const char *cache_path, void *stream, ws_tuning *out);
/* Autotuner of a batch: the same candidates timed on the batched kernels over
 * all attached domains (predictor and corrector passes, as above), applied
 * to the batch and returned.  Synchronous. */
ws_status ws_batch_tune(ws_batch *b, void *stream, ws_tuning *out);

/* Thread-local description of the last error. */
const char *ws_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
