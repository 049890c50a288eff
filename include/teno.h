/*
 * teno.h -- C-ABI of libteno.so: the TENO5-LAD semi-discrete Euler
 * right-hand side and its SSP-RK3 drivers on one MI355X (gfx950) GPU.
 *
 * Method: Peng, Li, Shen, Liu, Zhang, "An efficient targeted ENO scheme with
 * local adaptive dissipation for compressible flow simulation",
 * arXiv:2003.09145.
 *   - semi-discrete conservative form du/dt = -(f_{i+1/2} - f_{i-1/2})/dx,
 *     one direction at a time, summed over x, y, z           (Sec. 2, eq 2.2)
 *   - global Lax-Friedrichs flux splitting, reconstruction in characteristic
 *     space                                                    (Sec. 4)
 *   - fifth-order TENO reconstruction: candidate fluxes, Jiang-Shu
 *     smoothness indicators, tau_5, scale separation, cutoff  (Sec. 2,
 *     eq 2.4-2.15)
 *   - locally adaptive cutoff C_T = Lad(m), m = B_l + floor(theta (B_u-B_l)),
 *     theta = 1 / (1 + max_k chi~_k / H)                      (Sec. 3,
 *     eq 3.1-3.4)
 *   - SSP-RK3 time stepping and CFL time step                 (Sec. 4,
 *     eq 4.1-4.3, eq dt1, eq dt2)
 *   - Euler equations of an ideal gas                          (Sec. 4.2, eq 4.7)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Fields: FP64, structure of arrays, component-major, x fastest:
 *     U[c * ncell + (k * ny + j) * nx + i],  ncell = nx * ny * nz,
 * components c = rho, rho*u_x, [rho*u_y], [rho*u_z], E (ncomp = ndim + 2),
 * interior cells only (ghost cells are synthesised on chip).
 *
 * Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 * tensors); every other pointer is a host pointer.  The caller owns every
 * buffer.  Entry points that take a stream enqueue work on it and return
 * without synchronising; device-detected errors are reported through the
 * device control block (teno_ctrl.status).  Host-side validation failures
 * return TENO_ERR_ARG and enqueue nothing.  No exceptions cross the ABI.
 * `stream` is a hipStream_t (NULL = the default stream).
 */
#ifndef TENO_H_
#define TENO_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define TENO_OK 0
#define TENO_ERR_ARG 1          /* invalid argument; nothing was enqueued       */
#define TENO_ERR_DEVICE 2       /* a HIP call failed                            */
#define TENO_ERR_NONPHYSICAL 3  /* rho <= 0, p <= 0 or a non-finite value seen  */

/* Boundary types, applied at both ends of an axis (Sec. 4.1: periodic;
 * Sec. 4.2: zero-gradient; Sec. 4.2 eq 4.11: reflecting).  Three ghost cells
 * per side: periodic wrap; copy of the edge cell; mirror image with the
 * normal momentum negated. */
#define TENO_BC_PERIODIC 0
#define TENO_BC_TRANSMISSIVE 1
#define TENO_BC_REFLECTIVE 2
/* A fixed ghost state (only through teno_boundary below): the Dirichlet ends
 * of the Rayleigh-Taylor and double Mach reflection problems of Sec. 4.3. */
#define TENO_BC_FIXED 3

/* One end of an axis whose boundary may change along the boundary and in
 * time.  Its ghost cells take kind[0] where the split coordinate -- the cell
 * centre (i + 1/2) dx along axis split_axis, measured from the grid's low
 * corner, on the boundary line -- lies below split[0] + split[1] * t, and
 * kind[1] elsewhere (split_axis = -1: kind[0] everywhere).  A TENO_BC_FIXED
 * part supplies state[part] (conserved variables, natural order, ncomp used). */
typedef struct teno_side {
    int32_t kind[2];      /* TENO_BC_*                                            */
    int32_t split_axis;   /* 0, 1, 2, or -1                                       */
    int32_t reserved_;
    double split[2];      /* split position split[0] + split[1] * t               */
    double state[2][5];   /* fixed ghost states                                   */
} teno_side;

/* Per-end boundaries, a gravity source and the time of teno_rhs calls, in
 * DEVICE memory (read by the kernels).  Boundaries are evaluated at the
 * stage times t, t + dt, t + dt/2 of teno_step and at t_rhs by teno_rhs.
 * The source adds rho g_d to each momentum component and sum_d m_d g_d to
 * the energy after the flux differences (Sec. 4.3: rho and rho v for the
 * Rayleigh-Taylor problem, g = (0, 1)). */
typedef struct teno_boundary {
    teno_side side[3][2]; /* [axis][0: low end, 1: high end]                      */
    double gravity[3];
    double t_rhs;
} teno_boundary;

/* Cutoff schemes: the locally adaptive C_T (Sec. 3), a fixed C_T (TENO5,
 * Sec. 2 eq 2.14), or every stencil kept (the linear upwind scheme eq 2.3). */
#define TENO_SCHEME_LAD 0
#define TENO_SCHEME_FIXED_CT 1
#define TENO_SCHEME_LINEAR5 2
/* TENO5-A: the adaptive cutoff of Sec. 2 eq 2.16-2.18 (the paper's comparison
 * scheme), C_T = 10^-floor(beta) from the sensor eta of the reconstruction's
 * own five values. */
#define TENO_SCHEME_TENO5A 3

/* Grid, gas and scheme parameters (host struct, read at call time). */
typedef struct teno_grid {
    int32_t ndim;      /* 1, 2 or 3                                             */
    int32_t n[3];      /* cells per axis; axes >= ndim must be 1; n >= 3 on the
                          swept axes                                            */
    double dx[3];      /* uniform spacing per axis (> 0)                        */
    int32_t bc[3];     /* TENO_BC_* per axis                                    */
    int32_t scheme;    /* TENO_SCHEME_*                                         */
    double gamma;      /* ratio of specific heats (> 1), eq 4.7                 */
    double ct_fixed;   /* C_T of TENO_SCHEME_FIXED_CT                           */
    double H;          /* LAD intensity threshold, eq 3.2 (paper: 10)           */
    int32_t Bl, Bu;    /* LAD magnitude bounds, eq 3.1 (paper: 4, 10);
                          0 <= Bl <= Bu <= 20                                   */
    double eps;        /* epsilon of eq 2.8 and eq 3.2 (paper: 1e-6)            */
    int32_t flags;     /* TENO_FLAG_* (0 for normal use)                        */
    int32_t theta;     /* LAD theta form of eq 3.2: TENO_THETA_PRINTED (0) or
                          TENO_THETA_CUT (1); other schemes ignore it          */
    double a1, a2;     /* TENO5-A alpha_1, alpha_2 of eq 2.16 (paper: 10.5, 3.5);
                          0 <= a1 - a2, a1 <= 20                                */
    double cr;         /* TENO5-A C_r of eq 2.17 (paper: 0.25); 0 < 0.9 cr < 1  */
    double xi;         /* TENO5-A xi of eq 2.18 (paper: 1e-3); >= 0             */
    const teno_boundary* boundary_dev; /* nullable: per-end boundaries and gravity
                          (device memory); when set, bc[] is not used.  Not
                          supported by the adjoint and batched entry points
                          (TENO_ERR_ARG)                                        */
} teno_grid;

/* teno_grid.flags: evaluate every cutoff decision with the literal formula
 * instead of the certified fast path (identical results, slower; for
 * verification and timing comparisons). */
#define TENO_FLAG_LITERAL_DECISIONS 1
/* teno_grid.flags: teno_step launches the sweep variant that accumulates the
 * cutoff-mask digest into ctrl.digest while ctrl.want_digest is set.  Without
 * this flag the sweeps carry no digest code and ctrl.digest is left alone. */
#define TENO_FLAG_MASK_DIGEST 2

/* teno_grid.theta: the LAD sensor of eq 3.2, with x = max_k chi-tilde_k.
 * TENO_THETA_PRINTED: theta = 1 / (1 + x / H) as printed.
 * TENO_THETA_CUT: theta = 0 where x > H, the printed form elsewhere.  Sec. 3
 * describes H as the threshold above which the whole stencil counts as
 * discontinuous, and theta = 0 as the value of a discontinuity (C_T =
 * 10^-B_l); the printed form gives theta = 1/2 at x = H instead.  With H = 10
 * the cut form runs the double Mach reflection of Sec. 4.3.3 to t = 0.2,
 * which the printed form does not. */
#define TENO_THETA_PRINTED 0
#define TENO_THETA_CUT 1

/* Time-stepping control block.  Lives in DEVICE memory so that step loops
 * never synchronise with the host and can be captured in a HIP graph. */
typedef struct teno_ctrl {
    double t;            /* current time                                         */
    double t_end;        /* the step is clipped so that t never passes t_end     */
    double cfl;          /* CFL number sigma of eq dt1 / eq dt2                   */
    double dt;           /* dt of the last step (input in replay mode)           */
    double alpha[3][3];  /* LF speeds [stage][axis] used by the last step
                            (input in replay mode)                               */
    int32_t status;      /* sticky TENO_OK / TENO_ERR_NONPHYSICAL                */
    int32_t replay;      /* 0: dt and alpha from the state; 1: taken from here   */
    int64_t nsteps;      /* number of completed steps                            */
    int32_t active;      /* internal: 1 while the current step is running        */
    int32_t want_digest; /* 1: accumulate the cutoff-mask digest below            */
    uint64_t digest;     /* sum over every face of every stage of a 64-bit hash of
                            (nsteps, stage, axis, face, the 2*ncomp cutoff masks):
                            equal digests mean (with overwhelming probability)
                            identical masks at every face, stage and step         */
    uint64_t reserved_[2];
} teno_ctrl;

/* Bytes of device workspace that teno_rhs / teno_step / teno_rhs_adjoint need
 * for this grid (three state-sized buffers plus a small scratch area).
 * Returns 0 for an invalid grid. */
size_t teno_workspace_bytes(const teno_grid* g);

/* Fill a device control block: t = t0, t_end, cfl, replay = 0, status = OK,
 * nsteps = 0, want_digest = 0, digest = 0 (enqueued on `stream`). */
int teno_ctrl_init(teno_ctrl* ctrl_dev, double t0, double t_end, double cfl,
                   void* stream);

/* Prepare ctrl_dev to replay a recorded step: copy dt and alpha[3][3] from
 * recorded_dev (a control block saved after a teno_step), set replay = 1,
 * status = OK and t_end = +inf; t, nsteps and the digest fields of ctrl_dev
 * are kept (enqueued). */
int teno_ctrl_replay(teno_ctrl* ctrl_dev, const teno_ctrl* recorded_dev, void* stream);

/* Switch the cutoff-mask digest of later teno_step calls on (enable = 1) or
 * off, and reset it to 0 (enqueued).  Only grids with TENO_FLAG_MASK_DIGEST
 * accumulate it. */
int teno_ctrl_digest(teno_ctrl* ctrl_dev, int32_t enable, void* stream);

/* dUdt_dev = L(U_dev): the semi-discrete RHS of eq 2.2 summed over the axes
 * in the order x, y, z (dUdt = 0 - dF_x/dx - dF_y/dy - dF_z/dz), with
 * characteristic TENO5-LAD reconstruction of global Lax-Friedrichs split
 * fluxes (Sec. 2-4).
 *   alpha_in_dev   nullable: 3 doubles of frozen LF speeds per axis; when
 *                  null they are computed from U as max_i (|u_d| + c).
 *   alpha_out_dev  nullable: receives the speeds used (3 doubles).
 *   status_dev     nullable: int32, set to TENO_ERR_NONPHYSICAL if U has a
 *                  cell with rho <= 0, p <= 0 or a non-finite sound speed
 *                  (only checked when alpha is computed).
 *   ws_dev, ws_bytes  workspace of at least teno_workspace_bytes(g).
 * U_dev and dUdt_dev must not overlap. */
int teno_rhs(const teno_grid* g, const double* U_dev, double* dUdt_dev,
             const double* alpha_in_dev, double* alpha_out_dev,
             int32_t* status_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): L(U)
 * exactly as teno_rhs (the same kernels, bit-identical results), with no
 * workspace argument.  The LF-speed partials and the speeds in use live in a
 * fixed 72 KiB device array of the library, one copy per GPU, looked up on
 * the first call on each device and held until the process ends; the call
 * allocates nothing.  Its size does not depend on the grid, so every grid
 * teno_rhs accepts is accepted (invalid arguments: TENO_ERR_ARG, a failed
 * address lookup or launch: TENO_ERR_DEVICE).  All calls on one GPU share
 * that array: calls that overlap in time on one GPU (several streams or
 * threads) race and must be ordered by the caller. */
int teno_rhs_noalloc(const teno_grid* g, const double* U_dev, double* dUdt_dev,
                     const double* alpha_in_dev, double* alpha_out_dev,
                     int32_t* status_dev, void* stream);

/* As teno_rhs, and also writes the cutoff decisions of every scalar
 * reconstruction: per axis d (x, y, z), per line, per face phi = i + 1 in
 * [0, n_d], 2*ncomp bytes (characteristic field s, sign + then -), each byte
 * m | (mask << 5) with m the ladder exponent (0 unless LAD) and mask bit k =
 * delta_k of eq 2.14.  Lines of axis x are numbered k*ny + j, of axis y
 * k*nx + i, of axis z j*nx + i.  decisions_dev holds
 * sum_d (ncell / n_d) (n_d + 1) 2 ncomp bytes. */
int teno_rhs_debug(const teno_grid* g, const double* U_dev, double* dUdt_dev,
                   const double* alpha_in_dev, double* alpha_out_dev,
                   int32_t* status_dev, uint8_t* decisions_dev, void* ws_dev,
                   size_t ws_bytes, void* stream);

/* One direction of eq 2.2 (one sweep kernel launch):
 *   Rout = Rin - (F^_{i+1/2} - F^_{i-1/2}) / dx_axis      (Rin == NULL: 0),
 * with F^ the characteristic TENO5-LAD flux of global LF split fluxes using
 * alpha_dev[axis] (alpha_dev: 3 device doubles).  Rin may equal Rout (each
 * cell is read and written by one thread); U must not overlap Rout.  This is
 * the building block that teno_rhs launches once per axis. */
int teno_sweep(const teno_grid* g, int32_t axis, const double* U_dev,
               const double* Rin_dev, double* Rout_dev, const double* alpha_dev,
               void* stream);

/* Self-test of the device arithmetic the path relies on, for n inputs:
 * q[i] = a[i] / b[i] by the general routine and q2[i] = a[i] / b[i] by the
 * reciprocal-based routine of the hot loops, s[i] = sqrt(a[i]) -- all
 * correctly rounded (IEEE-754 binary64, round to nearest even) whenever
 * operands and results lie in [2^-900, 2^900] in magnitude -- and r[i] = the
 * approximate reciprocal of b[i] used by the decision fast path.  For
 * comparison, qplain[i] and splain[i] (both nullable) receive the compiler's
 * own a[i] / b[i] and sqrt(a[i]) with no correction, the operations the
 * correctly rounded routines replace.  All pointers are device pointers of
 * n doubles. */
int teno_selftest_arith(const double* a_dev, const double* b_dev, double* q_dev,
                        double* q2_dev, double* s_dev, double* r_dev,
                        double* qplain_dev, double* splain_dev, int64_t n, void* stream);

/* One SSP-RK3 step of eq 4.1-4.3, in place on U_dev:
 *   u1 = u + dt L(u);  u2 = 3/4 u + 1/4 u1 + 1/4 dt L(u1);
 *   u  = 1/3 u + 2/3 u2 + 2/3 dt L(u2),
 * with the LF speeds recomputed for every stage and dt from the speeds of u
 * (eq dt1 in 1D, eq dt2 in 2D, sigma / sum_d(alpha_d / dx_d) in 3D), clipped
 * so that t + dt <= t_end.  In replay mode (ctrl.replay = 1) dt and the
 * per-stage speeds are read from the control block instead.  The step is a
 * no-op when ctrl.status != OK or t >= t_end; a non-physical stage state sets
 * ctrl.status and leaves U_dev at its value before the step. */
int teno_step(const teno_grid* g, double* U_dev, teno_ctrl* ctrl_dev,
              void* ws_dev, size_t ws_bytes, void* stream);

/* teno_step with timing marks, for profiling the launches of a step inside a
 * longer timed region.  events: 2 * 3 * ndim hipEvent_t handles created by the
 * caller (entries may be null); events[2 * (ndim * s + d)] is recorded on
 * `stream` right before the sweep kernel of axis d in RK stage s and
 * events[2 * (ndim * s + d) + 1] right after it.  Results are identical to
 * teno_step. */
int teno_step_timed(const teno_grid* g, double* U_dev, teno_ctrl* ctrl_dev,
                    void* ws_dev, size_t ws_bytes, void* const* events, void* stream);

/* Graph-replayed time stepping (eq 4.1-4.3 with the time-step control of
 * teno_step).  A step never waits on the host -- dt, t and the status live
 * in the device control block -- so a run of steps can be recorded once as a
 * HIP graph and replayed: the host then submits one graph per
 * steps_per_graph steps instead of every kernel of every step.  (On a small
 * grid such as the 200-cell Sod tube the kernels' own device time, not the
 * host's launch work, sets the pace, so the replays gain little there.)
 *
 * teno_runner_create records steps_per_graph (1 .. 1000) consecutive
 * teno_step calls on (g, U_dev, ctrl_dev, ws_dev) into a graph.  The grid
 * description, the three device pointers and the workspace size are fixed
 * at creation: the runner is valid while they are unchanged, and must be
 * destroyed and re-created after any change to *g.  U_dev, ctrl_dev and
 * ws_dev stay owned by the caller; the runner owns its graph and a private
 * capture stream.  Returns TENO_ERR_ARG on an invalid grid, null pointer,
 * short workspace or steps_per_graph out of range, TENO_ERR_DEVICE on a HIP
 * error.
 *
 * teno_runner_run enqueues nsteps (>= 0) steps on `stream`: nsteps /
 * steps_per_graph replays of the graph followed by the remaining steps
 * launched one by one.  The result is bit-identical to nsteps teno_step
 * calls, including the clipping at ctrl.t_end (later steps are no-ops) and
 * the sticky status.  Runs on one runner must not overlap (they share U, the
 * control block and the workspace). */
typedef struct teno_runner teno_runner; /* opaque */
int teno_runner_create(const teno_grid* g, double* U_dev, teno_ctrl* ctrl_dev, void* ws_dev,
                       size_t ws_bytes, int32_t steps_per_graph, teno_runner** out);
int teno_runner_run(teno_runner* r, int64_t nsteps, void* stream);
int teno_runner_destroy(teno_runner* r);

/* ------------------------------------------------------------------------
 * Discrete adjoint.  With the cutoff flags delta_k of eq 2.14 (hence the
 * weights of eq 2.15) and the LF speeds held fixed, L is a smooth function of
 * U; these entry points apply the transpose of its Jacobian A(U) = dL/dU and
 * of one SSP-RK3 step.  The flags are recomputed from U with the forward
 * arithmetic, so they are exactly the forward pass's.
 *
 * What is differentiated is the fixed-step map: the time step dt_n and the
 * per-stage speeds alpha_{n,s} are inputs (recorded by the forward run), not
 * functions of U.  Both are maxima over cells of |u_d| + c, so they depend on
 * U only through the cell that attains the maximum; that derivative is not
 * included.  A finite-difference check must replay the recorded dt and
 * speeds (teno_ctrl_replay) to see the same map.
 * ------------------------------------------------------------------------ */

/* Workspace bytes for teno_rhs_adjoint / teno_step_adjoint: six state-sized
 * buffers and the per-chunk partial gradients of every axis (ncomp x 74
 * doubles per 64 faces when the line has 63 cells or more, about 1.16 states
 * per axis), which one gather pass sums.  0 for an invalid grid. */
size_t teno_adjoint_workspace_bytes(const teno_grid* g);

/* gradU_dev = A(U)^T lambda_dev with the LF speeds alpha_dev (3 device
 * doubles) frozen.  Deterministic (fixed summation order, no floating-point
 * atomics).  gradU must not overlap U or lambda. */
int teno_rhs_adjoint(const teno_grid* g, const double* U_dev, const double* alpha_dev,
                     const double* lambda_dev, double* gradU_dev, void* ws_dev,
                     size_t ws_bytes, void* stream);

/* Transpose of one SSP-RK3 step (eq 4.1-4.3) taken from state Un_dev with the
 * dt and per-stage speeds recorded in ctrl_dev (dt, alpha[3][3], as left by
 * the forward teno_step): the stage states are rebuilt with those frozen
 * values, then lambda_dev (cotangent of the step's output) is replaced in
 * place by the cotangent of Un:
 *   l2 = 2/3 l + 2/3 dt A(u2)^T l;   l1 = 1/4 l2 + 1/4 dt A(u1)^T l2;
 *   l <- 1/3 l + 3/4 l2 + l1 + dt A(u^n)^T l1. */
int teno_step_adjoint(const teno_grid* g, const double* Un_dev, const teno_ctrl* ctrl_dev,
                      double* lambda_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Scalar linear advection u_t + u_x = 0 (Sec. 4.1, eq 4.4) on a periodic 1D
 * grid (g->ndim = 1; bc is not used, no boundary_dev), with the scheme of g:
 * global Lax-Friedrichs splitting with alpha = 1 (f+ = u, f- = 0), each split
 * flux reconstructed at every face by the scalar TENO5 of Sec. 2-3 (f- on the
 * mirrored stencil), and the flux difference of eq 2.2.  The Table 1 test
 * and the approximate dispersion relation of the scheme use it.
 * ------------------------------------------------------------------------ */

/* Workspace bytes for teno_advect_step (three arrays of n doubles), 0 for an
 * invalid grid. */
size_t teno_advect_workspace_bytes(const teno_grid* g);

/* dudt_dev = -(F_{i+1/2} - F_{i-1/2}) / dx for u_dev (n doubles each, device,
 * not overlapping).  Enqueued on stream. */
int teno_advect_rhs(const teno_grid* g, const double* u_dev, double* dudt_dev, void* stream);

/* One SSP-RK3 step (eq 4.1-4.3) of size h >= 0, in place. */
int teno_advect_step(const teno_grid* g, double* u_dev, double h, void* ws_dev,
                     size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched form: nbatch independent 1D problems of uneven length, each with
 * its own LF speed, time step, time and status (the method of Sec. 2-4 per
 * problem).  Fields are packed component-major over the concatenated tubes:
 *     U[c * total + off_b + i],  off_b = sum of the lengths of tubes < b,
 * c = rho, rho*u, E.  One RK stage of every tube is one persistent kernel
 * launch; teno_batch_run replays a captured HIP graph of 10 steps.
 * ------------------------------------------------------------------------ */
typedef struct teno_batch_plan teno_batch_plan; /* opaque */

/* Build a plan (host call; allocates the plan's device tables and two stage
 * buffers of 3*total doubles).  g supplies gamma, the scheme parameters and
 * bc[0] (applied at both ends of every tube); its ndim/n/dx are ignored.
 * lengths[nbatch] >= 3 and dx[nbatch] > 0 are host arrays.  Every tube uses
 * CFL number cfl and stops at t_end (INFINITY: never).  tune_cache (nullable)
 * is a file of earlier autotuning results; a matching entry selects the
 * launch configuration. */
int teno_batch_plan_create(const teno_grid* g, int64_t nbatch, const int64_t* lengths,
                           const double* dx, double cfl, double t_end,
                           const char* tune_cache, teno_batch_plan** plan);
int teno_batch_plan_destroy(teno_batch_plan* plan);

/* Total number of cells (sum of the lengths), or -1 for a null plan. */
int64_t teno_batch_total_cells(const teno_batch_plan* plan);

/* Reset every tube to t = 0 and compute its LF speed from U_dev (enqueued). */
int teno_batch_init(teno_batch_plan* plan, const double* U_dev, void* stream);

/* One SSP-RK3 step (eq 4.1-4.3) of every tube, in place: 3 launches. */
int teno_batch_step(teno_batch_plan* plan, double* U_dev, void* stream);

/* nsteps steps; whole blocks of 10 steps are replays of a HIP graph captured
 * on the first call for this U_dev (the remainder is launched directly). */
int teno_batch_run(teno_batch_plan* plan, double* U_dev, int64_t nsteps, void* stream);

/* Pick the launch configuration (waves per block x persistent blocks per CU)
 * by timing `steps` steps of every candidate on a scratch copy of U_dev
 * (synchronous; allocates the scratch copy).  The result is appended to
 * tune_cache (nullable); an existing matching entry is used instead of
 * timing.  *best_ms (nullable) receives the best time per step, or -1 when
 * the cache was used.  The plan's per-tube state is unspecified afterwards:
 * call teno_batch_init. */
int teno_batch_autotune(teno_batch_plan* plan, const double* U_dev, int32_t steps,
                        const char* tune_cache, double* best_ms);

/* Current / explicit launch configuration (waves per block 1, 2 or 4;
 * persistent blocks per CU, 0 = one block per group of chunks). */
int teno_batch_get_config(const teno_batch_plan* plan, int32_t* waves,
                          int32_t* blocks_per_cu);
int teno_batch_set_config(teno_batch_plan* plan, int32_t waves, int32_t blocks_per_cu);

/* Copy the per-tube time, last dt, sticky status and step count to host
 * arrays of nbatch entries (each nullable); synchronises the device. */
int teno_batch_read(const teno_batch_plan* plan, double* t, double* dt, int32_t* status,
                    int64_t* nsteps);

#ifdef __cplusplus
}
#endif

#endif /* TENO_H_ */
