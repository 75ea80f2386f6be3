/*
 * ctuppm.h -- C ABI of the MI355X (gfx950) unsplit CTU/PPM hydro library.
 *
 * The calls follow the paper's statement of the problem: a block-structured
 * grid is a list of boxes per level, each box holding its conserved state with
 * ghost cells and handed to the compute kernels box by box (section 3; section
 * 4, the box iterator that passes each box's data pointer to a kernel); the
 * state advances one step at a time with dt from the CFL condition, using an
 * unsplit piecewise parabolic method (section 3.2); coarse and fine levels are
 * advanced with subcycling and then synchronised (section 3 and section 3.2).
 *
 * Conventions for every call:
 *   - All functions are extern "C", return an int status (CTUPPM_OK = 0, < 0 on
 *     error) and never throw; ctuppm_last_error() gives the message of the last
 *     failure on a context.
 *   - Every byte of device memory is the caller's (the Python binding
 *     allocates it with PyTorch): the state fabs and one workspace per
 *     problem.  The library keeps the raw pointers, never frees them and
 *     allocates no device memory.  Its device tables (the problem's records
 *     with dt, parity and counters, box records, work lists, ghost-fill and
 *     boundary tags, two-level tables) live at the start of the problem's
 *     workspace (ctuppm_workspace_meta_bytes() bytes, then the stage
 *     scratch) and are written by asynchronous copies on the context stream
 *     from pinned host staging buffers the context owns.
 *   - Work is enqueued asynchronously on the context's HIP stream (caller's);
 *     only ctuppm_get_dt, ctuppm_status, ctuppm_rejections,
 *     ctuppm_step_checked and ctuppm_stage_times synchronise it (and
 *     ctuppm_current_state after guarded steps).  Device buffers handed to the
 *     library must stay allocated until the stream has passed the last call
 *     that uses them (stream-ordered freeing, as PyTorch's allocator does on
 *     the same stream, is enough).
 *   - One context per host thread.
 *
 * State layout: one "fab" per box, FP64, [comp][k][j][i] over the box grown by
 * CTUPPM_NGHOST cells on every side, i fastest; components
 * (rho, rho u, rho v, rho w, rho E, rho X_1 .. rho X_nspec).  A box (nx, ny, nz)
 * has (5 + nspec)(nx+8)(ny+8)(nz+8) doubles.  Passive species are advected
 * with the flow (the paper's GPU proxy advects 13 species, section 4).  Each
 * box has two fabs, A and B; steps alternate between them and
 * ctuppm_current_state() tells which holds the current state.
 *
 * Schemes: the unsplit CTU/PPM advance (section 3.2), or the method-of-lines
 * formulation of the paper's GPU proxy (section 4): the same PPM parabolas
 * give the face states directly (edge values, no characteristic tracing, no
 * transverse corrections), HLLC fluxes give the flux divergence, and a
 * strong-stability-preserving Runge-Kutta method of order 2 or 3 advances the
 * state with a ghost fill before each stage.  Its dt uses the sum over
 * directions of the signal speeds.
 */
#ifndef CTUPPM_H
#define CTUPPM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CTUPPM_OK = 0,
  CTUPPM_EINVAL = -1,  /* bad argument (shapes, overlapping boxes, unknown id) */
  CTUPPM_ENOMEM = -2,  /* workspace smaller than ctuppm_workspace_bytes() */
  CTUPPM_EHIP = -3,    /* a HIP runtime call failed; see ctuppm_last_error */
  CTUPPM_ESTATE = -4,  /* call out of order (e.g. step before bind) */
  CTUPPM_ERETRY = -5   /* a step was rejected by the retry criterion; the current state is an
                          accepted one (U^n when nothing was committed) */
};
/* Physical boundaries, per side of each direction: periodic (both sides);
 * outflow (ghost cells copy the edge cell); reflecting wall (ghost cells
 * mirror the interior with the normal momentum negated, and every Riemann
 * problem on the wall face takes the mirror image of the inside state as the
 * outside state, so no mass crosses the wall); inflow (ghost cells hold
 * `inflow`, `inflow_X`). */
enum { CTUPPM_BC_PERIODIC = 0, CTUPPM_BC_OUTFLOW = 1, CTUPPM_BC_REFLECT = 2, CTUPPM_BC_INFLOW = 3 };
/* Step forms: one launch per stage per box; one persistent launch per stage
 * over the boxes of every problem stepped; the batched launches replayed from
 * a captured hipGraph; batched launches over waves of consecutive boxes (set
 * by ctuppm_set_wave_boxes, 64 by default) that share as many stage scratch
 * slots, so the workspace scales with the wave instead of the level (ghost
 * fill and the CFL pass still run over all boxes at once; single-level
 * problems). */
enum { CTUPPM_FORM_PER_BOX = 0, CTUPPM_FORM_BATCHED = 1, CTUPPM_FORM_GRAPH = 2, CTUPPM_FORM_WAVES = 3 };
/* Schemes: unsplit CTU/PPM; method of lines with SSP-RK2; with SSP-RK3. */
enum { CTUPPM_SCHEME_CTU = 0, CTUPPM_SCHEME_MOL_RK2 = 1, CTUPPM_SCHEME_MOL_RK3 = 2 };
/* Riemann solvers: HLLC (Toro, Spruce & Speares 1994, Davis speeds); the
 * two-shock approximate solver of the PPM lineage (Colella 1982; Colella &
 * Glaz 1985: both waves on shock curves, six Newton steps for the star
 * pressure, upwind sampling with a linear blend inside a straddling fan). */
enum { CTUPPM_RIEMANN_HLLC = 0, CTUPPM_RIEMANN_TWO_SHOCK = 1 };
/* PPM limiters: Colella & Woodward 1984 (eq. 1.10); the extremum-preserving
 * limiter of Colella & Sekora 2008 (smooth extrema keep their parabola). */
enum { CTUPPM_LIMITER_CW84 = 0, CTUPPM_LIMITER_CS = 1 };

#define CTUPPM_NVAR 5
#define CTUPPM_NGHOST 4

/* A box: inclusive valid cell range in its level's index space. */
typedef struct {
  int lo[3];
  int hi[3];
} ctuppm_box;

/* Problem parameters (level 0).  Level l has cell size dx / 2^l. */
typedef struct {
  double gamma;        /* ideal-gas ratio of specific heats, > 1 */
  double cfl;          /* Courant number: dt = cfl / max_cells max_d (|u_d|+c)/dx_d for CTU,
                          cfl / max_cells sum_d (|u_d|+c)/dx_d for the MOL schemes */
  double small_dens;   /* density floor */
  double small_pres;   /* pressure floor */
  double grav_z;       /* constant gravitational acceleration along z (0: none) */
  double dx[3];        /* level-0 cell size */
  int domain_lo[3];    /* level-0 index space of the domain, inclusive */
  int domain_hi[3];
  int bc_lo[3];        /* CTUPPM_BC_* per direction and side; periodic on both */
  int bc_hi[3];        /*   sides or neither */
  double inflow[5];    /* (rho, u, v, w, p) written by CTUPPM_BC_INFLOW */
  int nspec;           /* passive species (mass fractions) after rho E, 0..16 */
  int pad;
  double inflow_X[16]; /* species mass fractions written by CTUPPM_BC_INFLOW */
  int scheme;          /* CTUPPM_SCHEME_*; the MOL schemes are single-level */
  int riemann;         /* CTUPPM_RIEMANN_* */
  int limiter;         /* CTUPPM_LIMITER_* */
  int steepen;         /* 1: contact steepening of the density (CW84 section 1.3; with
                          CTUPPM_LIMITER_CW84 only) */
} ctuppm_params;

typedef struct ctuppm_ctx ctuppm_ctx;

/* Create a context that enqueues on `hip_stream` (a hipStream_t owned by the
 * caller; NULL = the null stream).  *out receives the context. */
int ctuppm_ctx_create(void* hip_stream, ctuppm_ctx** out);
/* Destroy a context, its problems, graphs and metadata tables. */
int ctuppm_ctx_destroy(ctuppm_ctx* ctx);
/* Message of the last error on ctx (static storage of the context). */
const char* ctuppm_last_error(ctuppm_ctx* ctx);

/* Define a problem (the box list of each level, section 3): nlevels (1 or 2;
 * refinement ratio 2), boxes[l] an array of nboxes[l] boxes of level l.  Boxes
 * of a level must not overlap, must lie in the level's domain, have edges of
 * at most 256 cells, and periodic domain extents must be >= CTUPPM_NGHOST.
 * The fine level is any set of disjoint boxes aligned to coarse cells (even
 * first and odd last indices), each at least 3 coarse cells inside the domain
 * (section 3 and its figure 1: fine boxes of several sizes, grouped in
 * several patches; section 3.2: subcycled levels synchronised by refluxing).
 * nspec must be 0..16, scheme a
 * CTUPPM_SCHEME_* value, riemann a CTUPPM_RIEMANN_* value, limiter a
 * CTUPPM_LIMITER_* value, and a two-level
 * problem uses CTUPPM_SCHEME_CTU (CTUPPM_EINVAL otherwise).  *pid_out
 * receives the id. */
int ctuppm_problem_create(ctuppm_ctx* ctx, const ctuppm_params* params, int nlevels,
                          const ctuppm_box* const* boxes, const int* nboxes, int* pid_out);
int ctuppm_problem_destroy(ctuppm_ctx* ctx, int pid);

/* Doubles in one fab of a box with nspec species: (5 + nspec)(nx+8)(ny+8)(nz+8)
 * (a box's state with its ghost cells, section 3).  CTUPPM_EINVAL for an
 * empty box or nspec outside 0..16.  Needs no context. */
int ctuppm_fab_elems(const ctuppm_box* box, int nspec, long long* elems);

/* Bytes of workspace a problem needs in a form: its device tables, the
 * Runge-Kutta stage fabs of the MOL schemes, the stage scratch (the batched
 * and graph forms hold every box's at once, the per-box form the largest
 * box's, the waves form one per box of a wave) and, with two levels, the
 * coarse region and the flux register (section 3.2).  The state of each box
 * is resident and handed over by pointer (section 4); this is the scratch the
 * advance needs beside it.  Depends on the boxes, nspec, the scheme and the
 * wave size, not on the tuning. */
int ctuppm_workspace_bytes(ctuppm_ctx* ctx, int pid, int form, size_t* bytes);
/* Bytes at the start of the workspace that hold the library's device tables
 * (the stage scratch follows).  Callers that poison or inspect the scratch
 * leave these bytes alone. */
int ctuppm_workspace_meta_bytes(ctuppm_ctx* ctx, int pid, size_t* bytes);

/* Hand the library the device pointers of level `level` (each box's resident
 * state, passed by pointer as in section 4): U_a[b], U_b[b] are the two fabs
 * of box b (CTUPPM state layout), 8-byte aligned, caller-owned.  The state is
 * taken to be in the A fabs (asynchronously: after the work enqueued before).
 * Nothing is changed when a pointer is null or misaligned (CTUPPM_EINVAL). */
int ctuppm_bind_state(ctuppm_ctx* ctx, int pid, int level, double* const* U_a, double* const* U_b);
/* Hand the library the problem's workspace (device, 256-byte aligned, at
 * least ctuppm_workspace_meta_bytes() bytes; CTUPPM_ENOMEM otherwise).  Its
 * first bytes receive the problem's device tables.  Re-binding a new
 * workspace moves the problem's records (parity, dt, counters) to it with an
 * asynchronous device copy, so the old workspace must stay allocated until the
 * stream has passed this call. */
int ctuppm_bind_workspace(ctuppm_ctx* ctx, int pid, void* workspace, size_t bytes);

/* Use a fixed dt (> 0) instead of the CFL time step; dt <= 0 restores CFL. */
int ctuppm_set_fixed_dt(ctuppm_ctx* ctx, int pid, double dt);

/* Advance each listed problem by one (coarse) step with its own dt: ghost
 * fill, dt from the CFL condition, cons->prim, flattening, PPM + tracing,
 * normal HLLC fluxes, the two transverse (CTU) stages, conservative update.
 * Two-level problems subcycle the fine level twice, then average down and
 * reflux.  MOL problems take their Runge-Kutta stages instead.  Problems
 * listed together must share one scheme, Riemann solver and limiter (CTUPPM_EINVAL
 * otherwise); a two-level problem steps on its own.  Asynchronous. */
int ctuppm_step(ctuppm_ctx* ctx, const int* pids, int npids, int form);

/* Guarded steps: the retry criterion of the paper's retry mechanism (section
 * 3.2, a step redone on criteria evaluated during the integration) checked on
 * the device.  Like ctuppm_step (single-level problems), but a problem whose
 * new state failed anywhere (a cell with rho < small_dens, p < small_pres or a
 * non-finite value, counter [4] of ctuppm_status) does not commit it: U^n stays
 * current (it is intact in the other fab) and the device counts a rejection,
 * which it also writes to host-mapped memory.  In the accepted case nothing
 * synchronises.  Returns CTUPPM_ERETRY, enqueuing nothing, when the host
 * already sees an unacknowledged rejection of a listed problem; the caller then
 * calls ctuppm_rejections (which acknowledges) and redoes the step with a
 * smaller dt (ctuppm_step_checked does that).  Steps enqueued after a rejected
 * one start again from U^n. */
int ctuppm_step_guarded(ctuppm_ctx* ctx, const int* pids, int npids, int form);
/* Rejected guarded steps of problem pid as the device has reported them so
 * far through host-mapped memory, without synchronising (exact for every
 * step whose completion the caller has observed, e.g. through an event
 * recorded after it); acknowledges them like ctuppm_rejections, but does not
 * update ctuppm_current_state's view of the parity. */
int ctuppm_rejections_seen(ctuppm_ctx* ctx, int pid, long long* rejected);
/* For callers that cannot allocate device memory at the time of the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): one step of a single-level problem as ctuppm_step takes it in
 * the batched form, with the stage scratch in the library's static device
 * array of CTUPPM_STATIC_SCRATCH_BYTES (one per GPU, held until the process
 * ends) instead of the workspace.  The caller still passes the state (bound
 * fabs) and a bound workspace, of which only the device tables and the MOL
 * stage fabs are used (a workspace bound for any form is enough; the tables
 * are uploaded when the state and the workspace are bound, CTUPPM_ESTATE if
 * they are not there).  Enqueues kernels only: no allocation, no copy, no
 * memset.  CTUPPM_EINVAL when the problem's stage scratch (every box's, as in
 * the batched form) exceeds CTUPPM_STATIC_SCRATCH_BYTES or it has two levels.
 * Every call on one GPU shares the array and leaves its contents behind
 * (nothing in it needs to start at zero); calls that overlap on one GPU, on
 * different streams or from different contexts, race. */
#define CTUPPM_STATIC_SCRATCH_BYTES (64u << 20)
int ctuppm_step_static(ctuppm_ctx* ctx, int pid);
/* Rejected guarded steps of problem pid so far (synchronises); acknowledges
 * them, so ctuppm_step_guarded accepts the problem again. */
int ctuppm_rejections(ctuppm_ctx* ctx, int pid, long long* rejected);
/* One step of a single-level problem with the retry mechanism (section 3.2):
 * a guarded step (synchronising for the verdict); if it is rejected, the
 * interval of the rejected dt is redone as two guarded steps of half of it,
 * and a rejected half again in two halves, down to an eighth of the dt.
 * *retried = the number of halvings the deepest retry used (0: accepted at
 * once).  CTUPPM_ERETRY when an eighth step is still rejected: the current
 * state is then the last accepted one (U^n if no part of the interval was
 * committed). */
int ctuppm_step_checked(ctuppm_ctx* ctx, int pid, int form, int* retried);
/* Test hook: the update flags one failed cell at step index step_index
 * (0-based count of accepted steps), -1 turns it off; a guarded step rejected
 * for it turns the hook off.  Forced from the host so every kernel still runs
 * to completion. */
int ctuppm_set_fail_hook(ctuppm_ctx* ctx, int pid, int step_index);

/* ------------------------------------------------------- a step in pieces
 * The paper states the problem a level at a time: fill the ghost cells of
 * every box, take dt from the CFL condition, advance each level with its
 * ghosts filled, then synchronise the levels -- average the fine level down
 * and reflux the coarse cells beside it (sections 3 and 3.2).  These calls
 * take one CTU step in those pieces, for callers that put their own work
 * between them (a dt reduced over several problems or devices, their own
 * boundary data, diagnostics).  Taken in the order below they give bitwise
 * the state ctuppm_step gives:
 *   single level:  fill_ghosts(0), compute_dt, advance_level(0)
 *   two levels:    fill_ghosts(0), compute_dt, advance_level(0),
 *                  { fill_ghosts(1), advance_level(1) } twice,
 *                  average_down, reflux
 * `form` is CTUPPM_FORM_PER_BOX, CTUPPM_FORM_BATCHED or CTUPPM_FORM_WAVES
 * (two-level problems: batched only); the graph form is ctuppm_step's.  The CTU scheme only (the
 * method-of-lines schemes fill ghosts inside their Runge-Kutta stages:
 * CTUPPM_EINVAL).  All calls are asynchronous on the context stream.  Calls
 * out of order return CTUPPM_ESTATE and enqueue nothing: advancing a level
 * whose current state has changed since its ghosts were filled, advancing
 * level 0 with no dt, a fine substep before the coarse advance or a third
 * one, averaging down before the second fine substep, refluxing before
 * averaging down; ctuppm_step, ctuppm_tag and ctuppm_regrid on a problem in
 * the middle of such a step. */

/* Ghost cells of level `level`'s current state: same-level copies (periodic
 * images included) and physical boundaries; on level 1 also the cells outside
 * the fine rectangle, interpolated from level 0 at the substep's time (after
 * the coarse advance: time fraction 0, then 1/2). */
int ctuppm_fill_ghosts(ctuppm_ctx* ctx, int pid, int level, int form);
/* dt of the next step from the CFL condition over the valid cells of every
 * level (two levels: the smaller of the coarse dt and twice the fine dt), or
 * the fixed dt; kept for the next advance and, when dt_dev is not NULL,
 * written to the device double *dt_dev. */
int ctuppm_compute_dt(ctuppm_ctx* ctx, int pid, int form, double* dt_dev);
/* Advance level `level` (ghost cells filled) by one step: cons->prim,
 * flattening, PPM + tracing, normal fluxes, both transverse stages, update.
 * Level 0 takes the dt of ctuppm_compute_dt, or the device double *dt_dev
 * when dt_dev is not NULL (the caller's dt, positive and finite, read on the
 * stream when the advance runs; a fine level then takes half of it); a
 * single-level problem's new state becomes current.  On two levels,
 * level 0 also records its fluxes on the coarse-fine faces and keeps its old
 * and new states for the fine ghost cells; level 1 (dt_dev NULL) takes half
 * the coarse dt and adds its fluxes to the register. */
int ctuppm_advance_level(ctuppm_ctx* ctx, int pid, int level, int form, const double* dt_dev);
/* Two levels, after the second fine substep: each coarse cell under the fine
 * rectangle becomes the average of its 8 children (section 3.2). */
int ctuppm_average_down(ctuppm_ctx* ctx, int pid);
/* Two levels, after averaging down: the coarse cells beside the fine
 * rectangle are corrected by the difference of the coarse flux and the summed
 * fine fluxes on their faces (refluxing, section 3.2); the new coarse state
 * becomes current and the step is complete. */
int ctuppm_reflux(ctuppm_ctx* ctx, int pid);

/* Which fab (0 = A, 1 = B) holds the current level-0 state of problem pid
 * (the state resident per box, section 4; the steps alternate between the two
 * fabs).  Synchronises after guarded steps, whose verdict only the device
 * knows. */
int ctuppm_current_state(ctuppm_ctx* ctx, int pid, int* which);
/* dt of the last step, from the CFL condition or the fixed dt (synchronises
 * the stream; CTUPPM_ESTATE before a workspace is bound). */
int ctuppm_get_dt(ctuppm_ctx* ctx, int pid, double* dt_host);
/* Counters (synchronises): [0] density floors, [1] pressure floors in
 * cons->prim, [2] floors on traced states, [3] transverse fall-backs,
 * [4] cells whose new state failed (rho < small_dens, p < small_pres or
 * non-finite: the criteria of the retry mechanism, section 3.2), [5] steps
 * committed.  All zero before a workspace is bound. */
int ctuppm_status(ctuppm_ctx* ctx, int pid, long long counters[6]);

/* Per-stage timing of eager launches: enable (1) or disable (0).  While on,
 * every stage launch of the per-box and batched forms is bracketed by HIP
 * events on the context stream. */
int ctuppm_set_timing(ctuppm_ctx* ctx, int on);
/* Accumulated milliseconds and launch counts per stage (synchronises), for
 * n <= ctuppm_num_stages() stages; resets the accumulators. */
int ctuppm_stage_times(ctuppm_ctx* ctx, double* ms, long long* launches, int n);
int ctuppm_num_stages(void);
const char* ctuppm_stage_name(int stage);

/* Algorithmic HBM bytes of one stage for one step of problem pid (each input
 * read once, each output written once, over that stage's regions), counting
 * every launch of the stage in a step of the batched form (the MOL schemes
 * run the fill, cons->prim, flattening, face-state, flux and update stages
 * once per Runge-Kutta stage). */
int ctuppm_stage_bytes(ctuppm_ctx* ctx, int pid, int stage, double* bytes);

/* ---------------------------------------------------------------- regridding
 * The paper's grids adapt: cells are tagged for refinement and boxes are built
 * around the tags (sections 2 and 3).  These calls tag, cluster and move the
 * fine level of a two-level problem. */

/* Tag the level-0 cells of problem pid whose density jumps across a cell in
 * some direction by more than `threshold` relative to the two neighbours:
 * |rho(i+e_d) - rho(i-e_d)| > threshold (rho(i+e_d) + rho(i-e_d)).  Fills the
 * current state's ghost cells first (valid cells are unchanged).  tags is a
 * caller-owned device array of nx*ny*nz bytes over the level-0 domain
 * (i fastest, 1 = tagged).  Asynchronous. */
int ctuppm_tag(ctuppm_ctx* ctx, int pid, double threshold, unsigned char* tags);

/* Berger & Rigoutsos (1991) clustering on the host: tags (host, nx*ny*nz
 * bytes, i fastest) are coarsened by `blocking` (a block is tagged if any of
 * its cells is), the blocks are clustered until each cluster's fraction of
 * tagged blocks reaches `efficiency` (0 < e <= 1) and no edge exceeds
 * `max_edge` cells (cuts at signature holes, then at the strongest inflection
 * of a signature, then across the middle of the longest edge), and the
 * clusters are refined back: boxes aligned to `blocking`, disjoint, covering
 * every tagged cell, clipped to the domain.  Writes at most `capacity` boxes;
 * *nboxes receives the count (CTUPPM_ENOMEM if it exceeds capacity).  Needs no
 * GPU. */
int ctuppm_cluster(const unsigned char* tags, const int n[3], int blocking, double efficiency, int max_edge,
                   ctuppm_box* boxes, int capacity, int* nboxes);

/* Replace the fine level of two-level problem pid by new boxes (the same
 * rules as in ctuppm_problem_create; for instance the boxes ctuppm_cluster
 * returns, scaled to the fine index space) with new caller-owned fabs Ua[b],
 * Ub[b].  The new fine state goes to Ua: cells under an old fine box are
 * copied from the old fine state, the others are interpolated conservatively
 * from the current coarse state (MC-limited linear, the coarse-fine ghost
 * interpolation at the start of a step).  Works in the stage scratch of the
 * bound workspace (which must hold the batched form's bytes).  Call between
 * steps; the old fabs may be freed once the stream has passed this call.  The
 * workspace must then be re-bound with ctuppm_workspace_bytes() bytes before
 * the next step (CTUPPM_ENOMEM otherwise).  Asynchronous. */
int ctuppm_regrid(ctuppm_ctx* ctx, int pid, const ctuppm_box* fine_boxes, int nfine, double* const* Ua,
                  double* const* Ub);

/* Graph form of single-level CTU steps: on, the captured step runs the three
 * directions of each phase (tracing + normal flux, first and second
 * transverse stage) on three streams, so the graph executes them
 * concurrently; off (default), one chain, which measures faster on the 256^3
 * workloads (the concurrent kernels share L2).  Results are the same either
 * way (each kernel writes its own arrays); graphs are re-captured. */
int ctuppm_set_concurrency(ctuppm_ctx* ctx, int on);
/* Debugging and stage-by-stage checks: copy one intermediate array of box
 * `box` of level `level`, as the last step taken in `form` left it in the
 * workspace, to the device buffer `out` (asynchronous; *elems receives its
 * length in doubles; out = NULL only reports the length).  Arrays: 0 the
 * primitives (rho, u, v, w, p, c, X_1..X_nspec) over the grown box; 1 the
 * flattening coefficient over cells -1..n; 2-4 the traced left states of the
 * x, y, z faces, 5-7 the right states (permuted primitives: density, normal
 * velocity, the two transverse velocities, pressure, species), 8-10 the
 * normal fluxes, 11-16 the first transverse-stage fluxes F^{A|B} (pair index
 * 2A + 0 for B = A+1, 2A + 1 for B = A+2, mod 3), 17-19 the final fluxes;
 * each halo-1 array is [component][k][j][i] over cells -1..n (a face array
 * holds face f of cell f's lower side), fluxes in global component order.
 * In the per-box form every box shares one scratch (the last box stepped);
 * in the waves form box b uses slot b mod the wave size.  The stage arrays
 * are the intermediates of the advance of section 3.2 (primitives, PPM face
 * states, Riemann fluxes of the unsplit corner transport); a two-level
 * problem takes the batched form only, and an array that would end past the
 * bound workspace is refused (CTUPPM_ENOMEM) without a copy. */
int ctuppm_debug_stage(ctuppm_ctx* ctx, int pid, int level, int box, int array, int form, double* out,
                       long long* elems);

/* Boxes per wave of CTUPPM_FORM_WAVES (>= 1); synchronises the context
 * stream.  Problems then need ctuppm_workspace_bytes(pid, CTUPPM_FORM_WAVES)
 * bytes: their MOL stage fabs plus min(boxes, number of boxes) slots of the
 * largest box's stage scratch. */
int ctuppm_set_wave_boxes(ctuppm_ctx* ctx, int boxes);

/* Kernels of the cell stages: on (1, the default), the flattening and the
 * tracing (CTU) or the edge-value face states (method of lines) of the three
 * directions run in one kernel that reads each cell's primitives once (the
 * passive species of the three directions follow in a kernel of their own,
 * stage "species_xyz", launched only for problems with species),
 * and the first transverse stage of the three directions (CTU) in one kernel
 * that reads each normal flux array once; 2, as 1 with the species traced
 * inside the merged kernels (no species stage); off (0), a flattening kernel
 * and one kernel per direction.  Results are the same bits in every mode
 * (each face takes the same arithmetic); captured graphs are dropped.
 * CTUPPM_EINVAL for another value. */
int ctuppm_set_fused(ctuppm_ctx* ctx, int on);
/* Measurement: the HBM bandwidth plain streaming reaches on this GPU, the
 * ceiling the stage kernels are compared with.  kind 0 copies `bytes` from src
 * to dst (counted read + write), 1 reads src, 2 writes dst; 16-byte accesses
 * in grid-stride loops, `reps` timed launches at each of a few grid sizes
 * (synchronises); *gbs receives the best rate in GB/s (1e9 bytes).  Buffers
 * are caller-owned device memory, 16-byte aligned, bytes a multiple of 16. */
int ctuppm_bandwidth_probe(ctuppm_ctx* ctx, int kind, const void* src, void* dst, size_t bytes, int reps,
                           double* gbs);
/* Tuning of the launches: blocks per CU of the persistent batched launches
 * (0 = one block per work unit), and the z planes one work unit marches
 * through in the batched/graph forms and in the per-box form (>= 1).  Results
 * do not depend on the tuning (each cell's arithmetic is the same); graphs are
 * re-captured and work lists rebuilt on the next step. */
int ctuppm_set_tuning(ctuppm_ctx* ctx, int blocks_per_cu, int zseg_batched, int zseg_per_box);
/* As ctuppm_set_tuning, plus the rows per tile the work units of a plane are
 * grouped into (0: the whole plane), which sets how far apart in the work list
 * a unit and its z neighbour are. */
int ctuppm_set_tuning2(ctuppm_ctx* ctx, int blocks_per_cu, int zseg_batched, int zseg_per_box, int ytile);
/* Per-stage tuning: the z planes one work unit of `stage` (an index below
 * ctuppm_num_stages()) marches through in the batched, graph and waves forms,
 * 1..64, multiplied by zseg_batched (the per-box form, whose launches cover
 * one box each, keeps one plane, two for cons->prim, times zseg_per_box).
 * Stages that run over the same work region share the setting:
 * ctuppm_stage_planes returns the stage's setting and its group (stages with
 * equal groups share it).  Defaults: 2 for cons->prim, 4 for the merged
 * tracing (and its species stage) and the merged method-of-lines face states,
 * 1 elsewhere.  Problems
 * stepped together whose merged-tracing work units at that depth would number
 * fewer than 8 per CU run their stages left at the defaults with one plane
 * per unit (two for cons->prim); a value set here is used as given.  Results
 * do not depend on it; work lists and graphs
 * are rebuilt on the next step.  CTUPPM_EINVAL for a stage without work units
 * (ghost fill, boundaries, dt, commit) or planes outside 1..64. */
int ctuppm_set_stage_planes(ctuppm_ctx* ctx, int stage, int planes);
int ctuppm_stage_planes(ctuppm_ctx* ctx, int stage, int* planes, int* group);

#ifdef __cplusplus
}
#endif
#endif
