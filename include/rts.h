/*
 * rts.h -- C ABI of librts, an MI355X (gfx950) short-characteristics radiation
 * transport solver (RTS) after arXiv 2107.08145 (MURaM), section "Summary of
 * the Radiation Transport Solver":
 *
 *   For every ray of a three-rays-per-octant angular quadrature and every
 *   frequency band, the transfer equation is integrated along short
 *   characteristics, upwind to downwind, plane by plane (the wavefront
 *   dependency figure: each point depends on up to four points of the previous
 *   plane).  Boundary intensities of the periodic horizontal directions are
 *   iterated a fixed number of times (the paper reports 3 to 4 iterations).
 *   The mean intensity J and the radiative heating Q are formed from the
 *   converged intensities (the "flux" step of the RTS core loop).
 *
 * Discretisation (shared with the CPU oracle by specification only):
 *   chi_b = kappa_b * rho;  dtau = ds/2 (chi_p + chi_u) with bilinear upwind
 *   values;  I_p = e I_u + w0 S_p + w1 S_u (S linear in tau), e = exp(-dtau);
 *   J_b = sum_r w_r I_r;  Q = sum_b qweight_b * 4 pi * chi_b * (J_b - S_b).
 *   Optional radiative flux vector (the flux step computes the mean intensity
 *   and the radiative fluxes from the same rays):
 *   F = sum_b qweight_b * 4 pi * sum_r w_r mu_r I_r, and its heating QF = -div F.
 *   The library sweeps D = I - S, an exact rewrite of the same recursion:
 *   D_p = e D_u + c (S_u - S_p), c = (1 - e)/dtau.
 *
 * Conventions
 *   - Arrays are C order [z][y][x], x fastest, k = 0 the bottom layer.
 *     N = nx*ny*nz.  Multi-band arrays are [band][z][y][x].
 *   - Array pointers in rts_inputs / rts_outputs / rts_seeds / rts_grads and the
 *     workspace are DEVICE pointers owned by the caller.  Pointers inside
 *     rts_desc (mu, w, qweight) are HOST pointers, read during
 *     rts_plan_create only.
 *   - The element type of kappa, rho, S, J, I_top, dS, dchi is double for
 *     RTS_FP64 and float for RTS_FP32; Q (and gQ) are always double.
 *   - All calls return an int status: RTS_OK (0) or a negative RTS_E_* code.
 *     No C++ exception crosses the ABI.  rts_status_string() describes a code;
 *     after RTS_E_HIP it also carries the HIP error text of the calling thread.
 *   - The library allocates no device memory.  Scratch space is the caller's
 *     workspace of at least rts_workspace_bytes() bytes, 256-byte aligned.
 *   - Work is enqueued on `hip_stream` (a hipStream_t, NULL = legacy default)
 *     and is asynchronous.  Outputs are overwritten, never accumulated.  For a
 *     fixed plan, results are bitwise reproducible.
 *   - A plan and its workspace must not be used by two calls in flight at the
 *     same time (they share the workspace's queue counters and flags).
 */
#ifndef RTS_H
#define RTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define RTS_OK 0
#define RTS_E_ARG (-1)         /* invalid argument: null pointer, bad size, mu_z == 0, ... */
#define RTS_E_UNSUPPORTED (-2) /* valid but not supported by the library (e.g. nx > 1024) */
#define RTS_E_WORKSPACE (-3)   /* workspace null, misaligned or too small                  */
#define RTS_E_HIP (-4)         /* a HIP runtime call failed                                */
#define RTS_E_DEADLOCK (-5)    /* the sweep's neighbour wait timed out (device status)     */
#define RTS_E_NOT_BUILT (-6)   /* no device code for the current GPU                       */
#define RTS_E_NONFINITE (-7)   /* an input holds a NaN or an infinity (rts_check_inputs)     */

typedef enum { RTS_FP64 = 0, RTS_FP32 = 1 } rts_precision;
/* Vertical boundaries (x and y are always periodic). */
typedef enum { RTS_BOT_THERMAL = 0 /* I = S */, RTS_BOT_FIXED = 1 /* I = i_bot */ } rts_bot_bc;
typedef enum { RTS_TOP_ZERO = 0 /* I = 0 */, RTS_TOP_THERMAL = 1 /* I = S */ } rts_top_bc;
/* Operations for rts_workspace_bytes. */
typedef enum { RTS_OP_SOLVE = 0, RTS_OP_ADJOINT = 1, RTS_OP_AUTOTUNE = 2 } rts_op;

typedef struct {
  int32_t nx, ny, nz; /* >= 2 each; nx, ny <= 1024 */
  double dx, dy, dz;  /* > 0 */
} rts_grid;

/* One box (one independent problem).  Paper: rays per octant, bands, boundary
 * iteration count and the radiative heating output ("Summary of the Radiation
 * Transport Solver"). */
typedef struct {
  rts_grid g;
  int32_t nbands;         /* >= 1 */
  int32_t nrays;          /* >= 1, <= 64 */
  const double* mu;       /* HOST [nrays][3]: unit direction vectors, mu_z != 0 */
  const double* w;        /* HOST [nrays]: quadrature weights, J = sum_r w_r I_r */
  const double* qweight;  /* HOST [nbands] or NULL (all 1): weight of band b in Q */
  int32_t bot;            /* rts_bot_bc, boundary of rays with mu_z > 0 (layer k = 0) */
  int32_t top;            /* rts_top_bc, boundary of rays with mu_z < 0 (layer k = nz-1) */
  double i_bot;           /* intensity for RTS_BOT_FIXED */
  int32_t n_iter;         /* >= 1: sweeps of rays whose dominant axis is x or y */
  int32_t prec;           /* rts_precision */
  int32_t flux;           /* 0 or 1: the workspace also holds flux partials per sweep task,
                             so that rts_solve / rts_solve_batched can write F and QF */
  double tol;             /* >= 0.  0: n_iter sweeps.  > 0: tolerance-driven boundary iteration
                             (the paper iterates boundary intensities until their error is
                             within a prescribed tolerance): the rays sharing an x or y dominant
                             axis and its direction sweep together until the largest change of
                             their outflow-plane intensities between successive sweeps is at
                             most tol times the largest outflow-plane intensity (the first sweep
                             compares with the initial ghost, I = S), n_iter sweeps at most.
                             Needs such a group to be one sweep task (at most four rays, one per
                             in-plane sign pattern, as S4): else RTS_E_UNSUPPORTED at
                             rts_plan_create.  rts_adjoint rejects it (RTS_E_UNSUPPORTED). */
  int32_t sub[3];         /* subdomain decomposition with lagged exchange (the paper's domain-
                             decomposed RTS: each subdomain integrates from the boundary
                             intensities its upwind neighbours produced in the previous
                             iteration, then passes its outflow intensities downstream).
                             All 0: the undivided solve above.  Else the box is cut into
                             sub[0] x sub[1] x sub[2] blocks along x, y, z (0 counts as 1; block
                             b of m along an axis of n cells holds cells [b n/m, (b+1) n/m),
                             1 <= sub[a] <= n along each axis), and every ray and band iterates
                             n_iter times: iteration k sweeps each block from iteration k's
                             values inside the block and iteration k-1's outside it (and for
                             the upwind plane of the block's first plane along the ray);
                             iteration 0 is I = S off the boundary layers.  With tol > 0 the
                             iterations stop after the first whose largest intensity change over
                             all cells, rays and bands of the box is at most tol times the
                             largest intensity.  One block (sub = {1,1,1}) is the undivided
                             solve with n_iter boundary iterations.  A plan's boxes are all
                             decomposed or none; a decomposed box has flux = 0 and no adjoint
                             (RTS_E_UNSUPPORTED). */
  int32_t gs_iter;        /* >= 0.  0: the source function S is given.  > 0: scattering, the
                             paper's Gauss-Seidel scheme for strongly scattering media (section
                             "RTS Integration and Interpolation Merge"): the source function is
                             S = (1 - eps) J + eps B, with B the `S` input (the thermal source)
                             and eps the photon destruction probability (rts_inputs.eps), and
                             gs_iter Gauss-Seidel iterations are run from S = B.  In one
                             iteration the ray groups (rays sharing the dominant axis and its
                             direction, in order of first appearance) sweep in turn with the
                             current S, the laps before a group's last iterating its periodic
                             boundary; in the last lap of the last group each point p is
                             updated as it is reached: with J' its mean intensity including the
                             group's new intensities and L(p) = sum_r w_r dI_r(p)/dS_p over every
                             ray, dS = ((1 - eps) J' + eps B - S) / (1 - (1 - eps) L(p)), S += dS,
                             and the group's intensities at p move by dI_r/dS_p dS before the
                             next points along the rays use them.  Q, J, I_top then come from the
                             last iteration (Q = sum_b qw_b 4 pi chi_b (J_b - S_b)) and
                             rts_outputs.S receives S.  Needs prec RTS_FP64, one box per plan,
                             flux = 0, tol = 0, no subdomains and one sweep task per dominant
                             axis and direction (at most four rays each, one per in-plane sign
                             pattern, as S4); else RTS_E_UNSUPPORTED.  No adjoint. */
} rts_desc;

typedef struct {
  const void* kappa; /* [nbands][N] opacity per unit mass */
  const void* rho;   /* [N] density */
  const void* S;     /* [nbands][N] source function (with desc.gs_iter > 0: the thermal source B) */
  const void* eps;   /* [nbands][N] photon destruction probability in (0, 1] for desc.gs_iter > 0
                        (required then, else ignored; may be NULL) */
  const void* ghost; /* warm start (the paper starts the boundary iteration from the previous time
                        step's intensities), or NULL (cold: I = S): the initial ghost-plane
                        intensities of every ray whose dominant axis is x or y,
                        [nbands][nrays][nz][max(nx, ny)]: the plane is the ray's outflow plane
                        (x = nx-1 or 0, y = ny-1 or 0 by its direction), row k its layer, column j
                        its y (x-dominant rays) or x (y-dominant rays) index; entries of
                        z-dominant rays and of the ray's boundary layer are not read.  Not with
                        subdomains, scattering or the adjoint (RTS_E_UNSUPPORTED); the element
                        type is the plan's. */
} rts_inputs;

typedef struct {
  double* Q;   /* [N] radiative heating, always written */
  void* J;     /* [nbands][N] mean intensity, or NULL */
  void* I_top; /* [nbands][n_up][ny][nx] intensity of the top layer for the n_up rays with
                  mu_z > 0 (in ray order), or NULL */
  double* F;   /* [3][N] flux vector (x, y, z components) sum_b qweight_b 4 pi sum_r w_r mu_r I_r,
                  or NULL; non-NULL needs the box's desc.flux (else RTS_E_ARG) */
  double* QF;  /* [N] heating -div F, or NULL; needs F: central differences, periodic in x and
                  y, second-order one-sided in the bottom and top layers (first-order if nz = 2) */
  void* S;     /* [nbands][N] the final source function of a scattering solve (desc.gs_iter > 0),
                  or NULL; ignored otherwise */
  void* ghost; /* the final ghost planes (each x or y dominant ray's outflow plane after its last
                  sweep), in the layout of rts_inputs.ghost, for the next call's warm start, or
                  NULL; must not alias rts_inputs.ghost.  Entries of z-dominant rays are not
                  written. */
} rts_outputs;

/* Adjoint seeds: L = <gQ, Q> + <gJ, J> + <gItop, I_top>; any may be NULL. */
typedef struct {
  const double* gQ;  /* [N] */
  const void* gJ;    /* [nbands][N] */
  const void* gItop; /* [nbands][n_up][ny][nx] */
} rts_seeds;

/* Adjoint results, overwritten: dL/dS_b and dL/dchi_b (chi_b = kappa_b * rho).
 * The caller applies dL/dkappa_b = rho dL/dchi_b, dL/drho = sum_b kappa_b dL/dchi_b. */
typedef struct {
  void* dS;   /* [nbands][N] */
  void* dchi; /* [nbands][N] */
} rts_grads;

/* Schedule knobs (chosen by the plan; settable for tuning). */
typedef struct {
  int32_t rows_per_strip; /* rows of the sweep plane per workgroup: 2, 4, 6 or 8 */
  int32_t max_workgroups; /* 0 = as many as are co-resident; never fewer than the strips of
                             the largest task (they must all be resident together) */
  int32_t order;          /* 0: longest sweeps first, 1: input order */
  int32_t use_graph;      /* 1: rts_solve and rts_solve_batched replay a captured hipGraph of
                             the whole call (re-captured when a pointer, the layout or the
                             timing switch changes) */
  int32_t single_launch;  /* 0: one persistent sweep launch per workgroup width (the sweep
                             tasks whose sweep planes round up to the same multiple of 64
                             columns), widest first, in stream order; 1: every task in one
                             launch as wide as the widest plane.  Forward results are
                             identical; adjoint gradients differ by rounding only (a task's
                             slot contributions are summed over as many partials as its
                             reverse launch has threads per column). */
  int32_t split_reverse;  /* accepted (0 or 1) and without effect: the adjoint's reverse sweep
                             always takes a task as two slot-pair passes (kept so that
                             schedules written for earlier versions stay valid) */
} rts_schedule;

/* Create a plan for `nbox` boxes (host only; validates every field; the
 * descs and their host arrays may be freed afterwards).  All boxes of one plan
 * share `prec`.  On success *out receives the plan. */
int rts_plan_create(const rts_desc* descs, int32_t nbox, void** out);

/* Bytes of device workspace needed by `op` (rts_op) on this plan: RTS_OP_SOLVE
 * for rts_solve / rts_solve_batched, RTS_OP_ADJOINT for rts_adjoint (it also
 * holds D of every plane of every ray group: at 128^3 with 24 rays and 3
 * iterations, 0.8 GB in FP32), RTS_OP_AUTOTUNE for rts_plan_autotune. */
int rts_workspace_bytes(void* plan, int32_t op, size_t* bytes);

/* Forward solve of box 0 of the plan (paper: the RTS call of one time step). */
int rts_solve(void* plan, const rts_inputs* in, const rts_outputs* out, void* ws,
              size_t ws_bytes, void* hip_stream);

/* Forward solve of all `nbox` boxes (nbox must equal the plan's box count):
 * every band, ray and box in one call, the sweep tasks of each workgroup width
 * in one persistent launch fed by a device-side work queue (one launch in all
 * with rts_schedule.single_launch); captured once into a hipGraph and replayed
 * when the schedule's use_graph is set. */
int rts_solve_batched(void* plan, int32_t nbox, const rts_inputs* in, const rts_outputs* out,
                      void* ws, size_t ws_bytes, void* hip_stream);

/* Reverse-mode gradients of L (rts_seeds) w.r.t. S and chi for every box of
 * the plan; `in`, `g`, `d` point to arrays of nbox entries; the workspace
 * must hold rts_workspace_bytes(RTS_OP_ADJOINT) bytes.
 *
 * This is the adjoint of the discrete forward solve (the recursion of the
 * "Summary of the Radiation Transport Solver" section as implemented by
 * rts_solve): the call re-runs the forward sweep, storing D of every plane
 * and lap in the workspace, then sweeps the transposed recursion downwind to
 * upwind in one persistent launch per workgroup width: every task as two
 * slot-pair passes (slots 0, 2 and 1, 3), strips of rows exchanging edge rows
 * with the one neighbour they depend on, recomputing the exp and
 * interpolation weights from chi and S and the upwind D from the cell's own
 * stored D.  Returns RTS_E_UNSUPPORTED if a box has tol > 0, for sweep planes
 * wider than 768 padded columns in FP64 (1024 in FP32), or if the strips of
 * one pass cannot all be resident (one workgroup per strip, at most one or
 * two per CU).  Seeds may be NULL (zero).  dS and dchi are
 * overwritten; chi = kappa * rho, so dL/dkappa_b = rho dL/dchi_b and
 * dL/drho = sum_b kappa_b dL/dchi_b.  Per-task partials are summed in a
 * fixed order in FP64: results are bitwise reproducible for a fixed plan. */
int rts_adjoint(void* plan, int32_t nbox, const rts_inputs* in, const rts_seeds* g,
                const rts_grads* d, void* ws, size_t ws_bytes, void* hip_stream);

/* The forward solve of all boxes (as rts_solve_batched, never from a graph)
 * that also keeps D of every plane and lap in the workspace, which must hold
 * rts_workspace_bytes(RTS_OP_ADJOINT) bytes, for a later
 * rts_adjoint_from_solve: the forward pass of a training step keeps what its
 * backward pass needs, as an autograd tape keeps activations.  Same errors as
 * rts_adjoint. */
int rts_solve_for_adjoint(void* plan, int32_t nbox, const rts_inputs* in, const rts_outputs* out,
                          void* ws, size_t ws_bytes, void* hip_stream);

/* rts_adjoint without its forward pass: the reverse sweep and the gradient
 * reduction read the D kept by the last rts_solve_for_adjoint on this
 * workspace, which the caller must leave untouched in between (no other call
 * of this plan on it) with the same inputs; the results are bitwise those of
 * rts_adjoint.  Seeds, gradients and errors as in rts_adjoint. */
int rts_adjoint_from_solve(void* plan, int32_t nbox, const rts_inputs* in, const rts_seeds* g,
                           const rts_grads* d, void* ws, size_t ws_bytes, void* hip_stream);

/* Autotuner: runs the forward solve of all boxes (as rts_solve_batched, not
 * replayed from a graph) under every candidate schedule -- rows per strip
 * 2/4/6/8 (FP32) or 2/4 (FP64), queue order 0/1, and single_launch 0/1 when
 * the sweep planes of the plan have more than one padded width -- `reps` timed calls each
 * after one warm-up call, timed with HIP events on `hip_stream`, and keeps
 * the fastest in the plan (written to *chosen if not NULL).  Candidates whose
 * workspace exceeds ws_bytes, or whose strips cannot all be resident, are
 * skipped; rts_workspace_bytes(RTS_OP_AUTOTUNE) covers every candidate.
 * Synchronous.  The choice is cached per process by problem shape and
 * device: a later call on an equal problem applies it without timing (and
 * leaves the outputs untouched).  When the environment variable
 * RTS_TUNE_CACHE names a file, that file is the cache instead, shared by
 * processes and runs: it is read on each call, keyed by the device's
 * architecture name, its compute-unit count and the problem (precision; per
 * box grid, bands, sweep tasks, sweeps and ray grouping), and each new choice
 * is appended as one text line "<key> <rows_per_strip> <order>
 * <single_launch>" (the last valid line of a key wins; lines that do not
 * parse or name no candidate schedule of the plan are ignored; a missing or
 * unwritable file only means no hit and no record).  Otherwise outputs hold
 * the result of the last timed call. */
int rts_plan_autotune(void* plan, int32_t nbox, const rts_inputs* in, const rts_outputs* out,
                      void* ws, size_t ws_bytes, void* hip_stream, int32_t reps,
                      rts_schedule* chosen);

/* For callers that cannot allocate device memory (code under hipGraph stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the forward
 * solve of all `nbox` boxes, as rts_solve_batched, with the library's own fixed
 * device array of RTS_STATIC_SCRATCH_BYTES bytes as its workspace instead of a
 * caller's.  Inputs and outputs are the caller's device pointers as above.
 *   - Limit: plans with rts_workspace_bytes(RTS_OP_SOLVE) above
 *     RTS_STATIC_SCRATCH_BYTES (64 MiB; at the default schedule 64^3 with 5
 *     bands in FP32 needs 49 MiB, 64^3 with 1 band in FP64 21 MiB) are refused
 *     with RTS_E_WORKSPACE before any device work.
 *   - The call allocates nothing: no device memory, no pinned host memory, no
 *     events or graphs.  It always runs eagerly (the schedule's use_graph and
 *     timing are ignored) and needs the plan's pinned task table, which
 *     rts_plan_create and rts_plan_set_schedule / rts_plan_autotune allocate
 *     when a GPU is visible (else RTS_E_UNSUPPORTED).
 *   - Each GPU holds one copy of the array from the library's first use on it
 *     until the process ends (its address is looked up once per device).  All
 *     calls on one GPU share it and it keeps the last call's contents (every
 *     call clears what must start at zero): two calls in flight on the same
 *     GPU at once, on any plans or streams, race and give wrong results.
 *     Serialise them (one stream, or events).
 *   - Results are bitwise those of rts_solve_batched with the same plan and
 *     schedule.  rts_check_status(plan, NULL, stream) reads the device status
 *     word the last call left in the array. */
#define RTS_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int rts_solve_static(void* plan, int32_t nbox, const rts_inputs* in, const rts_outputs* out,
                     void* hip_stream);

/* Optional input check, for callers that want non-finite inputs reported
 * rather than propagated (the solve itself does not test its inputs: a NaN
 * in chi or S spreads along the rays through every later plane and lap).
 * Scans every box's kappa [nbands][N], rho [N], S [nbands][N] and, for a
 * plan with desc.gs_iter > 0, eps [nbands][N] on the device, in the plan's
 * element type, for NaNs and infinities; the ghost planes are not scanned
 * (they may hold anything where they are not read).  Uses one status word
 * of `ws` (256-byte aligned, at least 256 bytes; the plan's solve workspace
 * will do, but not while a call of this plan is in flight on it), then
 * synchronises `hip_stream`.  Returns RTS_OK, RTS_E_NONFINITE, RTS_E_ARG
 * (null plan or inputs, nbox not the plan's, eps missing), RTS_E_WORKSPACE,
 * or a device error.  Reads each input once (at full HBM rate, about 0.2 ms
 * for five FP32 bands at 288^3). */
int rts_check_inputs(void* plan, int32_t nbox, const rts_inputs* in, void* ws, size_t ws_bytes,
                     void* hip_stream);

/* Synchronise `hip_stream` and read the device status word left in `ws` by
 * the last call: RTS_OK, or RTS_E_DEADLOCK if a neighbour wait timed out.
 * ws = NULL reads the status word of rts_solve_static's array on the current
 * device. */
int rts_check_status(void* plan, const void* ws, void* hip_stream);

int rts_plan_get_schedule(void* plan, rts_schedule* s);
int rts_plan_set_schedule(void* plan, const rts_schedule* s);

/* Device-side timing.  While enabled, each rts_solve / rts_solve_batched call
 * records HIP events on its stream around the sweep launches (one per
 * workgroup width, see rts_schedule.single_launch) and around the whole call
 * (up to 512 calls); a graph replay does so through event-record nodes of the
 * captured graph, re-pointed to the call's events before each replay.  rts_plan_last_timing waits for
 * the last recorded call and returns the mean sweep-kernel and whole-call
 * durations in ms over the calls recorded since timing was (re)enabled, or -1
 * if none.  Enabling resets the record. */
int rts_plan_enable_timing(void* plan, int32_t on);
int rts_plan_last_timing(void* plan, double* sweep_ms, double* total_ms);

void rts_plan_destroy(void* plan);
const char* rts_status_string(int status);
const char* rts_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RTS_H */
