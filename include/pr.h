/*
 * pr.h -- C ABI of the MI355X (gfx950) parareal-with-splitting library.
 *
 * Method: Arraras, Gaspar, Jimenez-Ciga, Portero, "Space-time parallel
 * iterative solvers for the integration of parabolic problems" (arXiv
 * 2502.08370). The library integrates the semi-discrete problem
 * U' = (A_1 + ... + A_M) U (section 2.2, eq. semidisc_prob) of the model
 * problem u_t = div(a grad u) - c u on the unit square / unit interval with
 * homogeneous Dirichlet data (section 2.1, eq. cont_problem, D = a I), using
 * the parareal algorithm (section 3) whose coarse propagator G and fine
 * propagator F are fractional implicit Euler (FIE, eq. FIE_method) under
 * dimensional splitting (A_1 = x-direction, A_2 = y-direction) or overlapping
 * domain-decomposition splitting with a partition of unity (section 2.1): in
 * 1D, components are intervals; in 2D, vertical strips (the subdomains of
 * Fig. fig:domaindecomposition), the partition of unity depending on x only.
 *
 * Discretisation: second-order finite differences on the interior nodes of a
 * uniform grid, h_x = 1/(nx+1), h_y = 1/(ny+1), diffusion coefficient given on
 * the cell faces (or as a nodal log-coefficient theta whose face value is the
 * mean of e^theta over the face's two nodes).
 *
 * Layouts (all FP64, all row-major with x fastest):
 *   state           U[j*nx + i], i in [0,nx), j in [0,ny) (ny = 1 in 1D)
 *   x-faces         ax[j*(nx+1) + f], face f between nodes f-1 and f
 *   y-faces         ay[g*nx + i], face g between nodes (i,g-1) and (i,g)
 *   nodal theta     theta[(j+1)*(nx+2) + (i+1)] with boundary nodes included
 *                   ((ny+2)*(nx+2) values; nx+2 values in 1D)
 *   PoU weights     1D DD: rho[k*(nx+1) + f], colour k, face f
 *                   2D DD: rho[k*(2*nx+1) + m], colour k, half-grid sample m
 *                   of x: m = 2f is x-face f, m = 2i+1 is node column i
 * A problem handle may hold several independent instances ("batch"); their
 * states are packed one after the other at the offsets pr_query_layout
 * returns.
 *
 * Pointers: every state / coefficient / gradient pointer is DEVICE memory
 * unless marked "host". hip_stream is a hipStream_t (NULL = default stream).
 * The caller owns every buffer it passes and keeps it alive until the work
 * queued on the stream has finished; the library owns its workspace
 * (factorisations, scratch, graphs), allocated in pr_create_problem and
 * released in pr_destroy_problem; no other call allocates device memory
 * except pr_parareal_iterate (its iteration graph, on first use) and
 * pr_adjoint (its recompute workspace of 2s+2 states plus N+1 checkpoints when
 * U_ckpt is NULL, on first use).
 *
 * Errors: every entry point returns a pr_status. Arguments are validated
 * before any work is queued: on PR_EINVAL / PR_EUNSUPPORTED nothing has been
 * written. HIP failures map to PR_EDEVICE, a NaN/Inf increment to
 * PR_ENUMERIC. pr_last_error() returns a thread-local message for the last
 * failure. No C++ exception crosses this interface. A handle must not be used
 * from two threads at once; distinct handles are independent.
 */
#ifndef PR_H
#define PR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pr_problem_s* pr_problem;

typedef enum {
  PR_OK = 0,
  PR_EINVAL = 1,        /* invalid argument or descriptor */
  PR_ENOMEM = 2,        /* device or host allocation failed */
  PR_EDEVICE = 3,       /* a HIP call failed */
  PR_ENUMERIC = 4,      /* NaN or Inf detected in a parareal increment */
  PR_EUNSUPPORTED = 5   /* valid request outside what the library implements */
} pr_status;

enum { PR_SPLIT_DIM = 0, PR_SPLIT_DD = 1 };          /* section 2.1 */
enum { PR_FIE = 0, PR_DR = 1 };                      /* eq. FIE_method, eq. DR_method */
enum { PR_COEF_FACES = 0, PR_COEF_NODAL_LOG = 1 };

/* Description of one problem instance (section 2.1, section 3).
 *   dim            1 or 2
 *   nx, ny         interior nodes per direction (ny must be 1 when dim == 1)
 *   T              final time (> 0)
 *   n_slices       N_c: coarse intervals, DT = T / N_c
 *   fine_steps     s: fine steps per coarse interval, dt = DT / s
 *   coarse_steps   FIE steps taken by one application of G (>= 1)
 *   fine           PR_FIE or PR_DR (the Douglas-Rachford fine propagator needs a
 *                  2D split; the coarse propagator is always FIE)
 *   split          PR_SPLIT_DIM (dim 2) or PR_SPLIT_DD (dim 1 or 2)
 *   coef_mode      PR_COEF_FACES: coef_x = ax, coef_y = ay (NULL in 1D)
 *                  PR_COEF_NODAL_LOG: coef_x = theta, coef_y unused
 *   coef_x, coef_y device pointers, read during pr_create_problem /
 *                  pr_set_coefficients only
 *   c              reaction coefficient >= 0; split equally over the M
 *                  dimensional terms (c/M per substep); weighted by rho_k in
 *                  the 2D DD terms; must be 0 for 1D DD
 *   n_colors       DD: number M of split terms (colours), 1..64
 *   rho            DD: HOST pointer to the partition-of-unity weights, each in
 *                  [0,1], summing to 1 at every sample (|sum - 1| <= 1e-14).
 *                  1D: [n_colors][nx+1] face weights; the components of colour
 *                  k are the maximal runs of faces with rho_k > 0, each one
 *                  independent tridiagonal system. 2D: [n_colors][2*nx+1]
 *                  samples on the half grid of x (x-fluxes take rho at their
 *                  face, y-fluxes and the reaction rho at the node column);
 *                  the strips of colour k are the maximal runs of columns with
 *                  rho_k > 0 on the node or on one of its x-faces, each one
 *                  independent 5-point system (at most 1024 columns wide),
 *                  solved exactly by block cyclic reduction in y with
 *                  precomputed w x w blocks: about 2.5 ny w^2 doubles of
 *                  device memory per strip and step size.
 *   n_forcing      number of separable source terms, 0..PR_MAX_FORCING: the
 *                  source of eq. FIE_method / eq. DR_method (homogeneous
 *                  boundary data) is F(t) = sum_m g_m(t) S_m, and tau F at the
 *                  step's end time enters the step's first stage
 *   forcing_space  device pointer, [n_forcing][ny][nx]: the grid functions S_m;
 *                  read during pr_create_problem only (the library keeps a copy)
 *   forcing_time_fine    HOST pointer, [n_forcing][n_slices * fine_steps]:
 *                  g_m at the end of fine step j of slice n, entry n*fine_steps + j
 *                  (t = n*DT + (j+1)*dt)
 *   forcing_time_coarse  HOST pointer, [n_forcing][n_slices * coarse_steps]:
 *                  g_m at the end of coarse step c of slice n (t = n*DT +
 *                  (c+1)*DT/coarse_steps)
 * Unused pointers may be NULL. */
#define PR_MAX_FORCING 2
typedef struct {
  int dim, nx, ny;
  double T;
  int n_slices, fine_steps, coarse_steps;
  int fine;
  int split;
  int coef_mode;
  const double* coef_x;
  const double* coef_y;
  double c;
  int n_colors;
  const double* rho;
  int n_forcing;
  const double* forcing_space;
  const double* forcing_time_fine;
  const double* forcing_time_coarse;
} pr_problem_desc;

/* Per-instance offsets (in doubles) into the packed buffers of a batch:
 *   u0_offset      single-state buffers (u0, grad_u0, lambda_T): npts each
 *   slices_offset  N-state buffers (pr_fine_propagate in/out, G_old): N*npts
 *   states_offset  (N+1)-state buffers (parareal iterate U): (N+1)*npts */
typedef struct {
  size_t u0_offset, slices_offset, states_offset;
  int npts, n_slices;
} pr_instance_layout;

/* Create a handle for n_instances problems (descs[0..n_instances-1], host
 * array). Validates every descriptor, allocates the workspace and computes
 * the per-line LU factorisations of I - tau A_j for tau = dt and tau = DT/
 * coarse_steps (section 2.2, eq. FIE_method), reading the coefficients on
 * hip_stream. *out receives the handle (NULL on failure). */
pr_status pr_create_problem(const pr_problem_desc* descs, int n_instances, void* hip_stream,
                            pr_problem* out);

/* Release the handle and its workspace (waits for the device). NULL is OK. */
pr_status pr_destroy_problem(pr_problem p);

/* Fill per_instance[0..n_instances-1] (host, may be NULL) and totals[3]
 * (host, may be NULL) = total doubles of the u0 / slices / states buffers. */
pr_status pr_query_layout(pr_problem p, pr_instance_layout* per_instance, size_t* totals);

/* Number of instances in the handle (host int). */
pr_status pr_num_instances(pr_problem p, int* n_instances);

/* Replace the diffusion coefficient of one instance (same coef_mode as at
 * creation; device pointers) and recompute its factorisations on hip_stream. */
pr_status pr_set_coefficients(pr_problem p, int instance, const double* coef_x,
                              const double* coef_y, void* hip_stream);

/* Fine propagator for all slices at once (section 3): F_out[n] = F^s(U_in[n])
 * for every instance and n = 0..N-1, each F^s being s FIE steps of size dt.
 * U_in and F_out use the slices layout and must not overlap. Asynchronous. */
pr_status pr_fine_propagate(pr_problem p, const double* U_in, double* F_out, void* hip_stream);

/* Coarse sweep of the parareal correction (section 3), serial in n:
 *   F == NULL (initial guess):  U[n+1] = G(U[n]),  G_old[n] = G(U[n])
 *   F != NULL (iteration):      g = G(U[n]); U[n+1] = F[n] + (g - G_old[n]);
 *                               G_old[n] = g
 * for n = 0..N-1 with U[0] left unchanged. U uses the states layout, F and
 * G_old the slices layout. inc_dev (device, n_instances doubles, may be NULL)
 * receives max_{n>=1} max_i |U_new[n]_i - U_old[n]_i| per instance (0 for the
 * initial guess; NaN/Inf propagate). Asynchronous. */
pr_status pr_coarse_sweep(pr_problem p, const double* F, double* G_old, double* U,
                          double* inc_dev, void* hip_stream);

/* Parareal (section 3): U[0] = u0, initial coarse guess, then corrections
 * until k_max corrections were done or the increment of an instance drops
 * below tol (instances that converged stop changing). u0 uses the u0 layout,
 * U the states layout (output: the final iterate). k_done and inc are HOST
 * arrays of n_instances entries: corrections performed and the last
 * increment. Each correction is one replay of a captured HIP graph followed
 * by one host synchronisation. Returns PR_ENUMERIC if an increment is NaN/Inf.
 * Reaching k_max with inc >= tol is not an error. */
pr_status pr_parareal_iterate(pr_problem p, const double* u0, double* U, int k_max, double tol,
                              int* k_done, double* inc, void* hip_stream);

/* Tuning options (pr_set_option / pr_get_option):
 *   PR_OPT_GRAPH       1 (default): pr_parareal_iterate captures one correction
 *                      as a HIP graph and replays it; 0: direct launches
 *   PR_OPT_FINE_CHUNK  chunk length of the fine line sweeps: 16, 20, 24, 32
 *   PR_OPT_TWISTED     1: each fine line is solved by two waves, one
 *                      eliminating from either end (twisted factorisation);
 *                      0: one wave per line. Default: 1 when one wave per line
 *                      would give fewer than 2048 waves per sweep over the
 *                      handle's instances, else 0; the default chunk is 20 when
 *                      the twisted lines include grouped ones (below), else 32
 *   PR_OPT_GROUPED     1 (default): with twisted sweeps, 64-slice blocks, the FIE
 *                      fine propagator and a chunk of 20 or 24, four lines per
 *                      workgroup share the loads of their pending-correction
 *                      carries through LDS; 0: one line per workgroup
 *   PR_OPT_LANES       slice lanes per line in the fine sweeps (lines per wave =
 *                      64 / lanes): 0 = per-instance default (the smallest power
 *                      of two >= N, in [8, 64]), or a cap of 8, 16, 32, 64
 *   PR_OPT_BLOCKS_PER_PASS  0 (default): every fine step covers all slice
 *                      blocks; k > 0: blocks are processed k at a time, each
 *                      group running all s fine steps before the next (a
 *                      smaller working set between consecutive sweeps)
 *   PR_OPT_PARTITIONED 1 (default): the fine sweeps of 2D FIE instances with
 *                      at most 24 slices whose lines fit one workgroup (at
 *                      most 1024 positions, and at most 8 * (64 / Lp) * 24
 *                      positions with slice blocks of Lp slices: few slices)
 *                      hold each line whole, cut into parts solved side by
 *                      side and joined exactly, and write exact values; for
 *                      those instances the options above then affect only the
 *                      adjoints' recomputed steps, which keep the chunked sweeps
 *                      (with more slices the chunked sweeps were measured faster);
 *                      2: every instance whose lines fit; 0: chunked sweeps
 *   PR_OPT_PARTITIONED_USED  read only (pr_set_option returns PR_EINVAL): the
 *                      number of the handle's instances whose fine sweeps are
 *                      partitioned under the current options
 * Results do not depend on the options beyond rounding. */
enum { PR_OPT_GRAPH = 1, PR_OPT_FINE_CHUNK = 2, PR_OPT_LANES = 3, PR_OPT_BLOCKS_PER_PASS = 4,
       PR_OPT_TWISTED = 5, PR_OPT_GROUPED = 6, PR_OPT_PARTITIONED = 7,
       PR_OPT_PARTITIONED_USED = 8 };
pr_status pr_set_option(pr_problem p, int option, int value);
pr_status pr_get_option(pr_problem p, int option, int* value);

/* Autotuner: times pr_fine_propagate on the handle's own shapes for every
 * (lanes, chunk, twisted) choice, keeps the fastest and reports it (host
 * pointers, each may be NULL; best_ms = its time; the twisted choice is read
 * with pr_get_option). Overwrites the library's internal
 * parareal buffers (not the caller's). Synchronous. */
pr_status pr_autotune(pr_problem p, void* hip_stream, int* lanes, int* chunk, float* best_ms);

/* Sequential fine solution (section 3, "fine approximation"): U[0] = u0,
 * U[n+1] = F^s(U[n]). u0: u0 layout, U: states layout. Asynchronous. */
pr_status pr_sequential_fine(pr_problem p, const double* u0, double* U, void* hip_stream);

/* Adjoint of the fine map u(T) = (F^s)^N u0 (dimensional splitting, FIE,
 * single-instance handles): for L = <lambda_T, u(T)>, writes
 * grad_u0 = dL/du0 (u0 layout) and grad_coef = dL/d(coefficient) in the
 * handle's coef_mode (faces: ax gradient followed by ay gradient; nodal log:
 * gradient with respect to theta, (nx+2)*(ny+2) values). U_ckpt (device,
 * states layout, may be NULL) receives the slice-boundary checkpoints of the
 * forward solve. Each FIE step is reversed with the transposed (= same,
 * symmetric) line solves in reverse substep order; the forward states inside
 * a slice are recomputed from its checkpoint. PR_EUNSUPPORTED for DD, 1D,
 * Douglas-Rachford or multi-instance handles. Asynchronous. */
pr_status pr_adjoint(pr_problem p, const double* u0, const double* lambda_T, double* grad_u0,
                     double* grad_coef, double* U_ckpt, void* hip_stream);

/* Allocation-free variant of pr_adjoint, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). Same arguments, outputs and restrictions as
 * pr_adjoint; instead of allocating its recompute workspace on first use it
 * carves it out of a fixed scratch array that every GPU the library runs on
 * holds for the life of the process (64 MiB = 8 Mi doubles; the device
 * address is taken per GPU by pr_create_problem). The workspace is
 * 2 s + 2 states, the two face-gradient arrays and, when U_ckpt is NULL, the
 * N + 1 slice-boundary checkpoints, each rounded up to 32 doubles: a problem
 * that needs more returns PR_EINVAL before any work is queued (pass U_ckpt to
 * fit a larger one). Calls the no-alloc entry point makes nothing else
 * allocate: the handle's own buffers come from pr_create_problem. Every call
 * on one GPU shares that GPU's array, so calls whose work overlaps on the
 * device (two streams, two threads) race; calls queued on one stream are
 * ordered. Asynchronous. */
pr_status pr_adjoint_noalloc(pr_problem p, const double* u0, const double* lambda_T,
                             double* grad_u0, double* grad_coef, double* U_ckpt,
                             void* hip_stream);

/* Parallel-in-time adjoint (not in the paper; derived from the transpose of
 * eq. FIE_method): same outputs as pr_adjoint. The adjoint of one slice's fine
 * map is the fine map of the transposed grid (each step: y solve, then x
 * solve), so the boundary adjoints lambda_n (lambda_N = lambda_T) are computed
 * as the states of the transposed problem, either exactly by its sequential
 * fine solve (k_max = 0) or by parareal on that backward problem (k_max > 0
 * corrections at most, stopping below tol; *k_done receives the count, host
 * pointer, may be NULL). Then every slice recomputes its forward steps and
 * runs its reverse steps at once, with the face gradients accumulated over
 * slices. Device workspace: two states per fine step per slice (2*s*N*nx*ny
 * doubles) plus small carries; PR_ENOMEM when it does not fit. Single
 * instance, 2D dimensional splitting, FIE fine propagator (else
 * PR_EUNSUPPORTED). Synchronizes hip_stream on entry; with k_max > 0 the call
 * is synchronous, otherwise the rest of the work is queued asynchronously. */
pr_status pr_adjoint_parallel(pr_problem p, const double* u0, const double* lambda_T,
                              double* grad_u0, double* grad_coef, double* U_ckpt, int k_max,
                              double tol, int* k_done, void* hip_stream);

/* Phase timers. When enabled, the library records a pair of hipEvents on the
 * work stream around every launch and accumulates their elapsed times per
 * phase (no extra synchronisation is added while recording). Phases:
 *   0 fine sweeps (one FIE substep of every line of every slice; a domain-
 *     decomposition colour substep counts as one)
 *   1 fine layout transposes (slice-interleaved workspace in/out)
 *   2 coarse x sweeps      3 coarse y sweeps (fused with the parareal update)
 *   4 other (copies, fills)
 *   5 whole coarse sweeps (span mode only)
 * pr_profile_control(p, 1) enables, 0 disables, 2 clears the totals, 3 enables
 * span mode: one event pair around each loop of fine sweeps (phase 0, counting
 * its launches) and each coarse sweep (phase 5, counting its slice steps)
 * instead of one per launch. Each event record costs a few microseconds of
 * queue time, so span mode is the one to use while timing whole iterations;
 * its per-launch means include the gaps between launches.
 * pr_profile_read waits for the recorded events and returns the totals. */
#define PR_PROFILE_PHASES 8
typedef struct {
  double ms[PR_PROFILE_PHASES];
  long long count[PR_PROFILE_PHASES];
} pr_profile;
pr_status pr_profile_control(pr_problem p, int mode);
pr_status pr_profile_read(pr_problem p, pr_profile* out);

/* Thread-local message describing the last non-OK status ("" if none). */
const char* pr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
