/*
 * burgers.h - C ABI of the MI355X (gfx950) viscous-Burgers steppers.
 *
 * Method: Potluri et al., "Explicit and implicit finite difference solvers implemented in JAX for
 * shock wave physics", arXiv 2601.12204.  The library advances batches of independent 1D viscous
 * Burgers problems u_t + u u_x = nu u_xx (eq. 1) on uniform grids with
 *   - the explicit forward-Euler step with first-order upwind convection and second-order central
 *     diffusion (Sec. 2.3, eq. 21; the upwind side follows the sign of u_i as the text after eq. 3
 *     describes), and
 *   - the implicit BTCS step (Sec. 2.4, eq. 23): the spatial operator at t^{n+1} with its convective
 *     coefficient lagged at u^n, i.e. one tridiagonal solve A(u^n) u^{n+1} = u^n per step, cyclic
 *     under periodic boundaries (eq. 18) and plain under Dirichlet boundaries (eqs. 16-17).
 *
 * Conventions shared by every entry point
 *   - Plain C types only; every pointer is either host memory (problem descriptions, offsets) or
 *     device memory on the context's device (states, gradients).  Device buffers are owned by the
 *     caller; the library never frees or reallocates them.
 *   - Packed layout: instance b occupies elements [off[b], off[b] + n_b) of a state buffer, with off
 *     from burgers_offsets().  Instance starts are aligned to BURGERS_ALIGN elements; the gaps are
 *     padding that the library neither reads for results nor writes.  A uniform batch whose n is a
 *     multiple of BURGERS_ALIGN is therefore plain row-major [count, n].
 *   - Element type is the context's dtype (IEEE binary32 or binary64), for every device buffer.
 *   - Calls enqueue work on the context's HIP stream and return without waiting.  Argument errors are
 *     reported synchronously and leave the state untouched.  Device errors are sticky: they are
 *     returned by the failing call if detected there, else by the next call or burgers_sync().
 *   - A context is not thread-safe.  Distinct contexts on distinct streams may be used concurrently.
 */
#ifndef BURGERS_H
#define BURGERS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BURGERS_ABI_VERSION 1
#define BURGERS_ALIGN 64 /* instance start alignment in elements */

typedef enum {
  BURGERS_OK = 0,
  BURGERS_E_INVALID = -1,     /* bad argument; nothing was enqueued */
  BURGERS_E_UNSUPPORTED = -2, /* valid request this build cannot serve (e.g. a forced path that
                                 does not fit the problem) */
  BURGERS_E_NOMEM = -3,       /* device allocation failed; the context stays usable */
  BURGERS_E_DEVICE = -4,      /* HIP runtime or kernel error (sticky) */
  BURGERS_E_NONFINITE = -5,   /* reserved: non-finite values reported by a checking call */
  BURGERS_E_BUDGET = -6,      /* reserved: request exceeds a memory budget */
  BURGERS_E_BOUND = -8,       /* reported by burgers_pool_retire: a truncated-window BTCS step of the
                                 slot failed its accuracy bound (far beyond the CFL step); pools do not
                                 redo such steps, so the state returned is not within the solver's
                                 accuracy: solve the problem through a context instead */
  BURGERS_E_NOT_CONVERGED = -7 /* reported by burgers_sync: since the last report, a Newton step
                                  (BURGERS_NEWTON) met a Jacobian row that was not strictly diagonally
                                  dominant, so its unpivoted solve was outside its stated range, or its
                                  last iteration's increment was not small against the iterate
                                  (1e-10 relative for binary64 states, 1e-5 for binary32); the states
                                  hold the iterates reached; the context stays usable */
} burgers_status;

typedef enum { BURGERS_BC_PERIODIC = 0, BURGERS_BC_DIRICHLET = 1 } burgers_bc; /* eq. 18; eqs. 16-17 */
/* Sec. 2.3 (forward Euler, eq. 21); Sec. 2.4 (BTCS, eq. 23); Sec. 2.7.1 (classical RK4, eq. 22, over
   eq. 21's spatial operator with the stages k1 = L(u), k2 = L(u + dt k1/2), k3 = L(u + dt k2/2),
   k4 = L(u + dt k3)); Crank-Nicolson, which Sec. 2.2 names beside BTCS: with the BTCS matrix written
   A = I + N (coefficients lagged at u^n), (I + N/2) u^{n+1} = (I - N/2) u^n; the fully implicit step
   with central convection of eqs. 10-14, F(u^{n+1}) = 0 solved by four Newton-Raphson iterations from
   u^n with the tridiagonal Jacobian of eq. 11 (no pivoting: meant for steps whose Jacobian stays
   strictly diagonally dominant, e.g. up to a few times the CFL step; every row is checked on the device
   and burgers_sync reports BURGERS_E_NOT_CONVERGED when one is not, or when the fourth increment is not
   at rounding level). */
typedef enum { BURGERS_EXPLICIT = 0, BURGERS_BTCS = 1, BURGERS_RK4 = 2, BURGERS_CN = 3,
               BURGERS_NEWTON = 4 } burgers_scheme;
typedef enum { BURGERS_F32 = 0, BURGERS_F64 = 1 } burgers_dtype;

/*
 * One problem instance (Sec. 2.2 and 2.5).
 *   n       stored grid nodes, 3 <= n <= 2^31 - 65536.  Periodic: nodes x_i = i*dx, dx = length/n, node n is
 *           node 0 again (eq. 18).  Dirichlet: dx = length/(n-1); nodes 0 and n-1 hold left and right
 *           (eqs. 16-17), and the n-2 interior nodes are the unknowns.
 *   length  domain length L > 0.
 *   nu      viscosity nu >= 0.
 *   dt      time step > 0.  The CFL limits (eqs. 7-8) are NOT enforced: the paper studies runs beyond
 *           them (Sec. 3.1); burgers_cfl_dt() computes a step inside them.
 *   bc      burgers_bc.    scheme  burgers_scheme (used by burgers_run and burgers_adjoint).
 *   left, right  Dirichlet values a, b; ignored for periodic instances.
 * The kernels use r = dt/dx and D = nu*dt/dx^2, computed once in binary64 on the host and rounded to
 * the working type.
 */
typedef struct {
  int64_t n;
  double length;
  double nu;
  double dt;
  int32_t bc;
  int32_t scheme;
  double left;
  double right;
} burgers_problem;

typedef struct burgers_ctx burgers_ctx; /* opaque */

/*
 * Kernel path selection.  0 means automatic (the library's tuned choice).  Forcing a path that cannot
 * serve some instance makes the stepping call return BURGERS_E_UNSUPPORTED.
 *   explicit_path  1 stream: one step per pass over HBM;
 *                  2 resident: a whole instance held on chip for many steps (n <= resident limit);
 *                  3 tiled: temporal blocking, tblock_depth steps per pass over HBM tiles.
 *   tblock_depth   steps per HBM pass of temporal blocking (1..512), 0 = automatic (128).
 *   btcs_path      1 workgroup: one workgroup solves one system per step (systems of up to 8192 rows,
 *                    or of exactly 16384: 1024 lanes of 16 rows; longer ones take btcs_long's solver);
 *                  2 resident: one workgroup per system for many steps;
 *                  3 multilevel: recursive partition across workgroups (any n).
 *   use_graph      1 replays the launch sequence of a stepping call from a captured HIP graph,
 *                  0 launches eagerly, -1 automatic.
 *   btcs_block     lanes per system for BTCS systems of exactly 8192 rows (512 lanes of 16 rows or
 *                  1024 of 8; 0 automatic = 512).  Systems of exactly 16384 rows take 1024 lanes of 16;
 *                  other whole systems the narrowest of 128, 256, 512 or 1024 lanes that holds them at
 *                  <= 8 rows per lane.
 *   btcs_long      solver of the other systems longer than 8192 rows (all but those of exactly 16384;
 *                  every BTCS and Crank-Nicolson step of them goes through HBM):
 *                  0 truncated windows (default): each window of 4096 rows (2: of 8192 rows, in
 *                    wider workgroups) is solved as a plain system
 *                    whose neighbours beyond its ends take their old values, and only its rows at least
 *                    256 rows inside are kept.  By the discrete maximum principle of the M-matrix
 *                    (strictly diagonally dominant rows, non-positive couplings) a kept row then differs
 *                    from the exact solution by at most 2^-54 max|u| whenever theta^257 <= 2^-56, with
 *                    theta = 2(D + C)/(1 + 2D + C + sqrt((1 + C)^2 + 4D)), C = r max|u| over the
 *                    window; every window checks this on the device each step, and an instance with a
 *                    window that fails it is solved again that step by the partition levels;
 *                  1 partition levels: the exact partition method across workgroups (three passes over
 *                    the state per step).
 *   serial         a call advances disjoint groups of instances: those held on chip (whole instances
 *                  of each scheme) and those stepped through HBM (explicit windows, per-step BTCS
 *                  solves).  0 (default): the groups run concurrently, on side streams of the context
 *                  forked from and joined back into its stream with events (parallel branches of a
 *                  captured graph); 1: one after another on the context's stream.
 *   btcs_pipeline  how the per-step path (btcs_path 1) solves systems of exactly 8192 rows: 1 persistent
 *                  workgroups, one per CU, each walking its share of the systems with the next system's
 *                  rows streaming into LDS while it solves the current one (systems whose first row is
 *                  16-byte aligned in 16-byte aligned state buffers, i.e. periodic ones; Dirichlet and
 *                  Crank-Nicolson systems keep one workgroup each); 2 one workgroup per system, several
 *                  per CU; 0 automatic (one workgroup per system, the faster on this GPU).  Both give
 *                  bitwise the same results.
 * burgers_set_plan rejects values outside these ranges with BURGERS_E_INVALID.
 */
typedef struct {
  int32_t explicit_path;
  int32_t tblock_depth;
  int32_t btcs_path;
  int32_t use_graph;
  int32_t btcs_block;      /* lanes for 8192-row BTCS systems: 512, 1024, or 0 = automatic */
  int32_t btcs_long;       /* systems of more than 8192 rows (other than 16384) stepped through HBM:
                              0 truncated windows of 4096 rows, 1 partition levels, 2 windows of 8192
                              rows (see below) */
  int32_t serial;          /* 1: one stream; 0: the independent launch groups run concurrently */
  int32_t btcs_pipeline;   /* per-step solves of exact 8192-row systems: 0 automatic, 1 persistent
                              workgroups that load the next system while solving one, 2 one workgroup
                              per system */
} burgers_plan;

/*
 * Create a context for `count` instances (count >= 1) of element type `dtype` whose work is enqueued
 * on `hip_stream` (a hipStream_t; NULL means the null stream) of the current device.  The problems
 * are copied; the context owns its workspace (a second state buffer for ping-pong stepping and the
 * solver's reduced systems), which is allocated here.
 * Errors: BURGERS_E_INVALID for a NULL pointer, count < 1 or an invalid problem (n < 3, length <= 0,
 * nu < 0, dt <= 0, bc or scheme out of range, any non-finite value); BURGERS_E_NOMEM when the
 * workspace cannot be allocated; BURGERS_E_DEVICE for a HIP failure.  *out is NULL on error.
 */
burgers_status burgers_create(const burgers_problem* problems, int64_t count, burgers_dtype dtype,
                              void* hip_stream, burgers_ctx** out);

/* Release the context and its workspace after draining its stream.  NULL is a no-op. */
void burgers_destroy(burgers_ctx* ctx);

/* Write the count+1 packed offsets (host array, elements) of the state layout into out. */
burgers_status burgers_offsets(const burgers_ctx* ctx, int64_t* out);

/* Number of elements a state buffer must hold (= the last offset). */
int64_t burgers_state_elems(const burgers_ctx* ctx);

/*
 * Advance every instance nsteps >= 0 explicit forward-Euler steps (Sec. 2.3, eq. 21, upwind side by
 * the sign of u_i), whatever its `scheme`.  u: device state buffer in the packed layout, updated in
 * place (the final state always lands in u).  Dirichlet nodes 0 and n-1 are set to left/right.
 * Rounding: binary64 states evaluate the same update as u_i + alpha (u_{i+1} - u_i) - beta (u_i - u_{i-1})
 * with beta = D + max(c_i,0), alpha = D - min(c_i,0), in fused multiply-adds (every execution path
 * gives bitwise the same result; over 10^4 CFL steps it stays within about 1e-13 of an unfused
 * evaluation of eq. 21, relative to max |u|); binary32 states round exactly as the unfused eq. 21.
 * Errors: BURGERS_E_INVALID (NULL ctx or u, nsteps < 0), BURGERS_E_UNSUPPORTED (forced path unfit),
 * BURGERS_E_DEVICE.
 */
burgers_status burgers_step_explicit(burgers_ctx* ctx, void* u, int64_t nsteps);

/*
 * Advance every instance nsteps >= 0 BTCS steps (Sec. 2.4, eq. 23): solve
 *   -(D + max(c_i,0)) u_{i-1} + (1 + 2D + |c_i|) u_i + (min(c_i,0) - D) u_{i+1} = u_i^n,
 * c_i = r u_i^n, for u^{n+1}; periodic systems are cyclic, Dirichlet systems carry the boundary values
 * on the right-hand side.  u as for burgers_step_explicit.  Errors as for burgers_step_explicit.
 */
burgers_status burgers_step_btcs(burgers_ctx* ctx, void* u, int64_t nsteps);

/*
 * Advance every instance nsteps >= 0 steps of its own `scheme` (forward-Euler, RK4 and BTCS instances
 * may be mixed in one context).  u as for burgers_step_explicit.  Errors as for burgers_step_explicit;
 * BURGERS_E_UNSUPPORTED also when RK4 instances meet a plan forcing explicit_path 1 (the one-step
 * streaming kernel is forward Euler only) or Crank-Nicolson or Newton instances meet btcs_path 2 (they
 * are solved per step through HBM: a Crank-Nicolson step is a BTCS solve with dt/2, y, followed by
 * u' = 2y - u; a Newton step is four assemble-solve-update iterations).
 */
burgers_status burgers_run(burgers_ctx* ctx, void* u, int64_t nsteps);

/*
 * As burgers_run, with separate step counts for the two kinds of scheme: instances whose `scheme` is
 * BURGERS_EXPLICIT or BURGERS_RK4 advance explicit_steps steps and the implicit ones (BURGERS_BTCS,
 * BURGERS_CN, BURGERS_NEWTON) btcs_steps steps (both >= 0), in one
 * launch sequence (one graph launch when use_graph is 1).  Ragged batches mixing schemes with
 * scheme-specific step budgets (explicit steps at the CFL limit, BTCS steps at a multiple of it) run
 * this way.  Errors as for burgers_step_explicit.
 */
burgers_status burgers_run_mixed(burgers_ctx* ctx, void* u, int64_t explicit_steps, int64_t btcs_steps);

/*
 * Discrete adjoint of burgers_run (the paper differentiates its solvers by reverse-mode AD, Sec. 2.7.1
 * and 2.7.3).  Given the initial state u0 and lambda_T = dJ/du(t_T) after nsteps steps of each
 * instance's scheme, write grad_u0 = dJ/du0 (packed layout) and grad_nu[b] = dJ/dnu_b (count values,
 * element type of the context).  Forward states are recomputed from checkpoints stored every
 * ckpt_every >= 1 steps: the context holds at most ceil(nsteps / ckpt_every) + 2 min(ckpt_every, nsteps) + 2
 * states of device memory (kept for later calls), and the results do not depend on ckpt_every, bit
 * for bit.  All four pointers are device memory; u0 and lambda_T are not modified.
 * Dirichlet boundary nodes are constants, so their entries of grad_u0 are zero.  The upwind switch is
 * differentiated on its u_i >= 0 branch at u_i = 0.
 * Errors: BURGERS_E_INVALID, BURGERS_E_NOMEM (checkpoint storage), BURGERS_E_DEVICE,
 * BURGERS_E_UNSUPPORTED (an FP32 context, or an RK4, Crank-Nicolson or Newton instance: the adjoint
 * covers forward Euler and BTCS).
 */
burgers_status burgers_adjoint(burgers_ctx* ctx, const void* u0, const void* lambda_T, int64_t nsteps,
                               int64_t ckpt_every, void* grad_u0, void* grad_nu);

/*
 * For callers that cannot allocate device memory (tight serving loops, harnesses that forbid hipMalloc):
 * burgers_run over a batch without a context.  Advances the `count` problems nsteps >= 0 steps of each
 * one's own scheme (as burgers_create + burgers_run + burgers_destroy would, with the same kernels and
 * results), enqueued on hip_stream of the current device, and returns without waiting.  u is the
 * caller's device state in the packed layout of burgers_offsets (instance starts aligned to
 * BURGERS_ALIGN elements), of element type dtype, updated in place.
 * Memory: the call allocates no device memory.  Its workspace (the instance and launch tables, the second
 * state buffer of ping-pong stepping and the reduced systems of long BTCS systems) lives in a static
 * device array of BURGERS_STATIC_SCRATCH_BYTES, one per GPU the library runs on, held until the process
 * ends.  Every call on a GPU reuses that GPU's array: calls on one stream are ordered, but calls that
 * overlap on one GPU (other streams, other threads) race and corrupt each other's results.  Nothing in
 * the array needs to start at zero.  Launches are eager (no graph).
 * Errors: BURGERS_E_INVALID (as burgers_create and burgers_run), BURGERS_E_BUDGET when the workspace
 * would exceed BURGERS_STATIC_SCRATCH_BYTES (nothing is run), BURGERS_E_UNSUPPORTED for Newton instances
 * (their checks report through burgers_sync of a context), BURGERS_E_DEVICE.
 */
#define BURGERS_STATIC_SCRATCH_BYTES (64u << 20)
burgers_status burgers_run_static(const burgers_problem* problems, int64_t count, burgers_dtype dtype,
                                  void* hip_stream, void* u, int64_t nsteps);

/*
 * Resident slot pools: continuous batching of solve requests (the serving workload of the paper's
 * solvers).  A pool holds `slots` device slots of one precision and one scheme (BURGERS_EXPLICIT or
 * BURGERS_BTCS), each able to hold a problem of up to max_nodes nodes (max_nodes <= 2^24), allocated
 * once at creation (two state buffers of slots x max_nodes elements when long problems fit, and the
 * slot tables).  Requests are admitted into free slots and retired between ticks; every tick advances
 * all occupied slots by up to tick_steps steps of their own problem in one launch sequence, replayed from
 * one of two HIP graphs (with and without the windows of long problems).  A slot runs exactly the kernels and arithmetic a
 * context holding its problem alone would run (on-chip whole instances up to 8192 nodes; explicit
 * windows or truncated BTCS windows beyond), so its result equals a burgers_run of the same problem,
 * except that a BTCS window whose accuracy bound fails is reported (BURGERS_E_BOUND) instead of redone.
 * All work is enqueued on hip_stream; a pool is not thread-safe.
 *
 * burgers_pool_create   Errors: BURGERS_E_INVALID, BURGERS_E_NOMEM, BURGERS_E_DEVICE.
 * burgers_pool_destroy  drains the stream and frees the pool (NULL is a no-op).
 * burgers_pool_admit    places problem p (scheme equal to the pool's, n <= max_nodes) with initial
 *                       state u0 (n values of the pool's precision, host or device memory; a host
 *                       buffer must stay unchanged until the stream has passed this call) and nsteps >= 1
 *                       steps to run into slot *slot (on entry: a free slot's index, or -1 for the lowest
 *                       free slot; on return: the slot used, -1 on error).  Errors: BURGERS_E_INVALID,
 *                       BURGERS_E_UNSUPPORTED (too long for the pool), BURGERS_E_BUDGET (the slot, or
 *                       every slot, is occupied), BURGERS_E_DEVICE.
 * burgers_pool_tick     enqueues one tick; each occupied slot advances min(tick_steps, its remaining
 *                       steps) steps.  Returns at once.
 * burgers_pool_busy     1 while the last enqueued tick has not finished, else 0.
 * burgers_pool_remaining  steps the slot has still to run (0: finished, awaiting retirement; -1: free;
 *                       -2: bad arguments).
 * burgers_pool_retire   enqueues a copy of a finished slot's state (n values) to dst (host or device) and
 *                       frees the slot.  Returns BURGERS_E_BOUND if one of its truncated-window steps
 *                       failed the accuracy bound (the copy is still made), BURGERS_E_INVALID for a slot
 *                       that is not finished.
 */
typedef struct burgers_pool burgers_pool;
burgers_status burgers_pool_create(burgers_dtype dtype, int32_t scheme, int64_t slots, int64_t max_nodes,
                                   int64_t tick_steps, void* hip_stream, burgers_pool** out);
void burgers_pool_destroy(burgers_pool* pool);
burgers_status burgers_pool_admit(burgers_pool* pool, const burgers_problem* p, const void* u0, int64_t nsteps,
                                  int64_t* slot);
burgers_status burgers_pool_tick(burgers_pool* pool);
int32_t burgers_pool_busy(burgers_pool* pool);
int64_t burgers_pool_remaining(const burgers_pool* pool, int64_t slot);
burgers_status burgers_pool_retire(burgers_pool* pool, int64_t slot, void* dst);

/* Wait for the context's stream and return the first sticky device error, if any; else
   BURGERS_E_NOT_CONVERGED once if a Newton check failed since the last report (see burgers_status). */
burgers_status burgers_sync(burgers_ctx* ctx);

/* Read or force the kernel path selection (see burgers_plan). */
burgers_status burgers_get_plan(const burgers_ctx* ctx, burgers_plan* out);
burgers_status burgers_set_plan(burgers_ctx* ctx, const burgers_plan* plan);

/*
 * Autotuner.  Times candidate plans on a scratch copy of the device state u (u itself is not modified)
 * for explicit_steps / btcs_steps steps (as burgers_run_mixed), with HIP events on the context's
 * stream, and keeps the fastest plan in the context.  It tunes one knob at a time, each over its values
 * with the others at their best so far, and only the knobs that matter for the context's instances:
 * the explicit path and, when some instance exceeds the on-chip limit, the temporal-blocking depth of
 * its windows (4, 8, 16, 32, 64, 128, 256 steps per pass over HBM); the lanes per 8192-row BTCS system
 * (512, 1024); the solver of BTCS systems longer than 8192 rows (truncated windows of 4096 or 8192 rows,
 * or the partition levels: the crossover between one-pass windows and the three-pass partition method);
 * concurrent launch groups on or off; and graph replay on or off.  Each candidate runs twice and the
 * second run is timed.  *best (optional) receives the chosen plan and *best_ms (optional) its time.  The
 * call synchronises the stream and allocates one scratch state, released before it returns.
 * Errors: BURGERS_E_INVALID, BURGERS_E_NOMEM, BURGERS_E_DEVICE.
 */
burgers_status burgers_autotune(burgers_ctx* ctx, const void* u, int64_t explicit_steps, int64_t btcs_steps,
                                burgers_plan* best, double* best_ms);

/* Static text for a status code. */
const char* burgers_status_string(burgers_status status);

/*
 * Time step inside the CFL limits of eqs. 7-8 with safety factor sigma:
 *   dt = sigma * min(dx / umax, dx^2 / (2 nu)),
 * dx from p->n, p->length and p->bc (p->dt is ignored).  A zero umax or nu drops that limit; returns
 * +inf when both are zero and NaN for an invalid p or sigma <= 0.  With sigma = 0.5 the step satisfies
 * |C| + 2D <= 1, the condition under which every explicit update is a convex combination.
 */
double burgers_cfl_dt(const burgers_problem* p, double umax, double sigma);

/* r = dt/dx and D = nu dt/dx^2 of a problem, in binary64, exactly as the kernels receive them. */
burgers_status burgers_ratios(const burgers_problem* p, double* r, double* D);

/* ABI version of the loaded library (BURGERS_ABI_VERSION at build time). */
int32_t burgers_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BURGERS_H */
