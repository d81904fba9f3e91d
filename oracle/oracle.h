/*
 * Oracle for the parareal-with-splitting hot path: a plain, serial, FP64 CPU
 * implementation written from the paper (Arraras, Gaspar, Jimenez-Ciga,
 * Portero, "Space-time parallel iterative solvers for the integration of
 * parabolic problems", arXiv 2502.08370).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The product path (the
 * HIP library under paper_2502_08370_amd/) never calls it and shares no code,
 * header, table or helper with it.
 *
 * Conventions (section 2, eq. semidisc_prob):
 *  - Unit square (or unit interval when dim == 1), homogeneous Dirichlet data,
 *    interior nodes only. h_x = 1/(nx+1), h_y = 1/(ny+1).
 *  - A grid function is stored row-major U[j*nx + i], x fastest, i in [0,nx),
 *    j in [0,ny). Node (i,j) sits at ((i+1)h_x, (j+1)h_y).
 *  - Face coefficients. ax[j*(nx+1) + f] is the diffusion coefficient on the
 *    x-face f of row j, between nodes f-1 and f (f = 0 and f = nx touch the
 *    boundary). ay[g*nx + i] is the y-face g of column i, between nodes
 *    (i,g-1) and (i,g).
 *  - Domain decomposition, 1D: rho[k*(nx+1) + f] is the partition of unity
 *    weight of colour k on face f. 2D (vertical strips, rho depends on x
 *    only): rho[k*(2*nx+1) + m] samples colour k's weight on the half grid of
 *    x, m = 2f on x-face f and m = 2i+1 at node column i.
 *  - Source term (F of eq. FIE_method and eq. DR_method, homogeneous boundary
 *    data): F(t) = sum_m g_m(t) S_m with n_forcing spatial factors S_m (grid
 *    functions) and g_m given at the time levels the steps use: fine step j of
 *    slice n ends at t = n*DT + (j+1)*dt (table entry n*fine_steps + j), coarse
 *    step c at t = n*DT + (c+1)*DT/coarse_steps (entry n*coarse_steps + c).
 *
 * All floating-point work is IEEE double, round to nearest, compiled with
 * contraction disabled so results are reproducible.
 */
#ifndef PR_ORACLE_H
#define PR_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int dim;            /* 1 or 2 */
  int nx, ny;         /* interior nodes; ny = 1 when dim == 1 */
  double T;           /* final time */
  int n_slices;       /* N_c, coarse step DT = T / N_c */
  int fine_steps;     /* s, fine step dt = DT / s */
  int coarse_steps;   /* FIE steps inside one coarse propagator call */
  int split;          /* 0: dimensional splitting, 1: domain decomposition */
  int fine_method;    /* 0: FIE, 1: Douglas-Rachford */
  double c;           /* linear reaction coefficient (not used by the 1D DD split) */
  const double* ax;   /* ny*(nx+1) x-face coefficients */
  const double* ay;   /* (ny+1)*nx y-face coefficients, NULL when dim == 1 */
  int n_colors;       /* domain decomposition: number of split terms M */
  const double* rho;  /* domain decomposition: n_colors*(nx+1) (1D) or
                         n_colors*(2*nx+1) (2D) partition of unity samples */
  int n_forcing;            /* separable source terms; 0: F = 0 */
  const double* fS;         /* n_forcing*nx*ny spatial factors S_m */
  const double* fg_fine;    /* n_forcing*(n_slices*fine_steps) values g_m */
  const double* fg_coarse;  /* n_forcing*(n_slices*coarse_steps) values g_m */
} or_problem;

/* Face coefficients a_f = (e^theta_p + e^theta_q)/2 from a nodal log
 * coefficient theta on the (nx+2)*(ny+2) grid that includes boundary nodes. */
void or_faces_from_theta(int nx, int ny, const double* theta, double* ax, double* ay);

/* 1D version: theta has nx+2 nodal values (boundary nodes included). */
void or_faces_from_theta_1d(int nx, const double* theta, double* ax);

/* Apply the full semi-discrete operator A = sum_j A_j (eq. semidisc_prob). */
void or_apply_A(const or_problem* p, const double* U, double* out);

/* Apply one split operator A_j (j = 0 x-direction / colour 0, ...). */
void or_apply_Aj(const or_problem* p, int j, const double* U, double* out);

/* One FIE step (eq. FIE_method) with step tau and source F (NULL: F = 0), in place. */
void or_fie_step(const or_problem* p, double tau, const double* F, double* U);

/* One Douglas-Rachford step (eq. DR_method) with step tau and source F (NULL: F = 0), in place. */
void or_dr_step(const or_problem* p, double tau, const double* F, double* U);

/* Fine propagator F^s over coarse interval n (its source levels), in place. */
void or_fine(const or_problem* p, int n, double* U);

/* Coarse propagator G over coarse interval n, in place. */
void or_coarse(const or_problem* p, int n, double* U);

/* F^s applied independently to n states U_in[n*npts] -> F_out (state k is
 * propagated over coarse interval k). */
void or_fine_batch(const or_problem* p, int n, const double* U_in, double* F_out);

/* Sequential fine solution at the coarse nodes: U[0] = u0,
 * U[n+1] = F^s(U[n]). U holds (N+1)*npts doubles. */
void or_sequential_fine(const or_problem* p, const double* u0, double* U);

/* One coarse sweep of the parareal correction (section 3).
 * F == NULL: initial guess U[n+1] = G(U[n]), G_old[n] = G(U[n]).
 * F != NULL: U[n+1] <- F[n] + (G(U[n]) - G_old[n]), G_old[n] <- G(U[n]),
 *            serially in n, U[0] unchanged. Returns the increment
 *            max_{n>=1} max |U_new[n] - U_old[n]| (0 for the initial guess). */
double or_coarse_sweep(const or_problem* p, const double* F, double* G_old, double* U);

/* Parareal (section 3): initial guess, then iterations until k_max
 * corrections are done or the increment drops below tol. U holds (N+1)*npts
 * doubles on return (iterate k_done). inc_hist[k] is the increment of
 * correction k+1. Returns k_done. */
int or_parareal(const or_problem* p, const double* u0, int k_max, double tol, double* U,
                double* inc_hist);

/* Gradient of L = <lambda_T, u(T)> through the sequential fine map
 * u(T) = (F^s)^N u0 (dimensional splitting, FIE). Outputs the gradient with
 * respect to u0 and to every face coefficient. */
void or_adjoint(const or_problem* p, const double* u0, const double* lambda_T, double* grad_u0,
                double* grad_ax, double* grad_ay);

/* Chain rule from face gradients to the nodal log coefficient theta. */
void or_theta_grad(int nx, int ny, const double* theta, const double* grad_ax,
                   const double* grad_ay, double* grad_theta);

#ifdef __cplusplus
}
#endif
#endif
