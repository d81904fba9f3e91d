/*
 * Oracle for the parareal-with-splitting hot path (arXiv 2502.08370).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path. Serial, FP64,
 * written for reading, not for speed: every substep assembles its tridiagonal
 * matrix from the operator definition and solves it with the textbook Thomas
 * algorithm.
 *
 * Paper passages followed (section / equation labels of the paper):
 *  - model problem and operator L u = div(D grad u) - c u: section 2.1,
 *    eq. cont_problem;
 *  - dimensional splitting L_j u = (d_jj u_{x_j})_{x_j} - c u / M: section 2.1;
 *  - domain decomposition splitting L_j u = div(rho_j D grad u) - rho_j c u with
 *    a partition of unity rho_j: section 2.1 (eq. partition_unity_M2 and the
 *    sub-operator definition after it);
 *  - method of lines U' = (A_1 + ... + A_M) U: section 2.2, eq. semidisc_prob;
 *  - fractional implicit Euler: section 2.2, eq. FIE_method;
 *  - Douglas-Rachford: section 2.2, eq. DR_method;
 *  - coarse/fine meshes, propagators, initial guess and the parareal
 *    iteration: section 3 (the displayed iteration after the initial guess);
 *  - adjoint: not in the paper; the transpose of the FIE step map, derived in
 *    the comment above or_adjoint.
 *
 * Readings where the paper is silent (all recorded in the design notes):
 *  - second-order finite differences on the interior nodes of a uniform grid,
 *    h = 1/(n+1) per direction, coefficient sampled on cell faces;
 *  - x substep first, then y; domain-decomposition colours in index order;
 *  - 2D domain decomposition: rho_j depends on x only (vertical strips) and is
 *    applied where each flux lives (x-faces for x-fluxes, node columns for
 *    y-fluxes and the reaction);
 *  - the parareal correction is evaluated as F_n + (G_new - G_old).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static double hx_of(const or_problem* p) { return 1.0 / (p->nx + 1); }
static double hy_of(const or_problem* p) { return 1.0 / (p->ny + 1); }
static int npts_of(const or_problem* p) { return p->nx * p->ny; }
static int n_terms(const or_problem* p) { return p->split == 1 ? p->n_colors : p->dim; }

/* Thomas algorithm (LU without pivoting) for a tridiagonal system with
 * sub-diagonal lo[i] (row i, column i-1; lo[0] unused), diagonal di[i] and
 * super-diagonal up[i] (row i, column i+1; up[n-1] unused). The right-hand
 * side x is overwritten with the solution. cp is scratch of length n. */
static void thomas(int n, const double* lo, const double* di, const double* up, double* x,
                   double* cp) {
  double piv = di[0];
  cp[0] = (n > 1) ? up[0] / piv : 0.0;
  x[0] = x[0] / piv;
  for (int i = 1; i < n; i++) {
    piv = di[i] - lo[i] * cp[i - 1];
    cp[i] = (i < n - 1) ? up[i] / piv : 0.0;
    x[i] = (x[i] - lo[i] * x[i - 1]) / piv;
  }
  for (int i = n - 2; i >= 0; i--) x[i] = x[i] - cp[i] * x[i + 1];
}

/* Scratch for one line of length n: sub, diag, super, pivot ratios, rhs. */
typedef struct {
  double *lo, *di, *up, *cp, *rhs;
} line_ws;

static line_ws ws_alloc(int n) {
  line_ws w;
  double* base = (double*)malloc(sizeof(double) * 5 * (size_t)(n > 0 ? n : 1));
  w.lo = base;
  w.di = base + n;
  w.up = base + 2 * n;
  w.cp = base + 3 * n;
  w.rhs = base + 4 * n;
  return w;
}
static void ws_free(line_ws* w) { free(w->lo); }

/* Assemble the matrix I - tau*A_line for one line of n nodes with face
 * coefficients face[0..n] (face f between nodes f-1 and f), spacing h and a
 * diagonal reaction term react >= 0 (so the row reads
 * -w_f u_{f-1} + (1 + w_f + w_{f+1} + tau*react) u_f - w_{f+1} u_{f+1},
 * w = tau*a/h^2). Faces 0 and n couple to Dirichlet boundary nodes (value 0). */
static void assemble_line(int n, const double* face, long face_stride, double h, double tau,
                          double react, line_ws* w) {
  for (int i = 0; i < n; i++) {
    double aw = face[(long)i * face_stride];
    double ae = face[(long)(i + 1) * face_stride];
    double ww = tau * aw / (h * h);
    double we = tau * ae / (h * h);
    w->lo[i] = -ww;
    w->up[i] = -we;
    w->di[i] = 1.0 + ww + we + tau * react;
  }
}

/* Domain decomposition in 2D (section 2.1, Fig. fig:domaindecomposition:
 * subdomains made of vertical strips). The partition of unity of colour j is
 * sampled on the half grid of x: r[2f] on x-face f (between nodes f-1 and f),
 * r[2i+1] at node column i. A_j discretises div(rho_j D grad u) - rho_j c u
 * with rho_j taken where each flux lives: x-fluxes at the x-faces, y-fluxes
 * (which sit at the node's x) at the node column, the reaction at the node.
 * Entry of row (i,k) of I - tau A_j; returns the diagonal, and the couplings
 * to the west, east, south and north neighbours through the out-pointers. */
static double dd2_row(const or_problem* p, const double* r, double tau, int i, int k, double* w,
                      double* e, double* so, double* no) {
  const int nx = p->nx;
  const double hx = hx_of(p), hy = hy_of(p);
  const double fw = r[2 * i] * p->ax[(long)k * (nx + 1) + i] / (hx * hx);
  const double fe = r[2 * i + 2] * p->ax[(long)k * (nx + 1) + i + 1] / (hx * hx);
  const double fs = r[2 * i + 1] * p->ay[(long)k * nx + i] / (hy * hy);
  const double fn = r[2 * i + 1] * p->ay[(long)(k + 1) * nx + i] / (hy * hy);
  *w = -tau * fw;
  *e = -tau * fe;
  *so = -tau * fs;
  *no = -tau * fn;
  return 1.0 + tau * (fw + fe + fs + fn + r[2 * i + 1] * p->c);
}

/* A column takes part in colour j's operator when rho_j is nonzero on its
 * node or on one of its two x-faces; otherwise its rows are identity rows. */
static int dd2_active(const double* r, int i) {
  return r[2 * i] > 0.0 || r[2 * i + 1] > 0.0 || r[2 * i + 2] > 0.0;
}

/* Banded LU without pivoting, in place: A[q][bw + (col - q)] holds the row's
 * band; the multipliers of L replace the entries they eliminate. */
static void band_lu(double* A, long n, long bw) {
  const long width = 2 * bw + 1;
  for (long q = 0; q < n; q++) { /* eliminate column q below the diagonal */
    const double piv = A[q * width + bw];
    const long last = (q + bw < n - 1) ? q + bw : n - 1;
    for (long t = q + 1; t <= last; t++) {
      const double f = A[t * width + bw + (q - t)] / piv;
      A[t * width + bw + (q - t)] = f;
      if (f == 0.0) continue;
      for (long c = q + 1; c <= q + bw && c < n; c++)
        A[t * width + bw + (c - t)] = A[t * width + bw + (c - t)] - f * A[q * width + bw + (c - q)];
    }
  }
}

/* Solve with the factors of band_lu, in place on b. */
static void band_solve(const double* A, long n, long bw, double* b) {
  const long width = 2 * bw + 1;
  for (long t = 1; t < n; t++) { /* forward: L y = b */
    const long first = t - bw > 0 ? t - bw : 0;
    double v = b[t];
    for (long q = first; q < t; q++) v = v - A[t * width + bw + (q - t)] * b[q];
    b[t] = v;
  }
  for (long q = n - 1; q >= 0; q--) { /* back substitution: U x = y */
    double v = b[q];
    for (long c = q + 1; c <= q + bw && c < n; c++) v = v - A[q * width + bw + (c - q)] * b[c];
    b[q] = v / A[q * width + bw];
  }
}

/* (I - tau A_j) V = U in place. Columns outside colour j's support are
 * identity rows and no x-face couples a supported column to an unsupported
 * one, so the system splits into one 2D system per maximal run of supported
 * columns (a strip, a connected component of the subdomain). Each strip system
 * is assembled in natural order (x fastest inside the strip, unknown
 * k*w + (i - i0)), which makes it banded with half-bandwidth w, and solved by
 * Gaussian elimination without pivoting (the matrix is a strictly diagonally
 * dominant M-matrix) followed by back substitution. The substep is an exact
 * solve; a direct solve in FP64 is accurate only to about the strip system's
 * condition number (1 + 8 tau max(a) / h^2, thousands at the paper's sizes)
 * times the unit roundoff, so the solution is improved by one step of
 * iterative refinement whose residual b - (I - tau A_j) x is accumulated in
 * extended precision (long double): x += solve(residual). */
static void dd2_substep(const or_problem* p, int j, double tau, double* U) {
  const int nx = p->nx, ny = p->ny;
  const double* r = p->rho + (long)j * (2 * nx + 1);
  int i0 = 0;
  while (i0 < nx) {
    if (!dd2_active(r, i0)) {
      i0++;
      continue;
    }
    int i1 = i0;
    while (i1 < nx && dd2_active(r, i1)) i1++;
    const int w = i1 - i0;
    const long n = (long)w * ny, bw = w, width = 2 * bw + 1;
    double* A = (double*)calloc((size_t)(n * width), sizeof(double)); /* A[q][bw + (col - q)] */
    double* b = (double*)malloc(sizeof(double) * n);
    double* x = (double*)malloc(sizeof(double) * n);
    for (int k = 0; k < ny; k++)
      for (int i = i0; i < i1; i++) {
        const long q = (long)k * w + (i - i0);
        double cw, ce, cs, cn;
        A[q * width + bw] = dd2_row(p, r, tau, i, k, &cw, &ce, &cs, &cn);
        if (i > i0) A[q * width + bw - 1] = cw;
        if (i + 1 < i1) A[q * width + bw + 1] = ce;
        if (k > 0) A[q * width + bw - w] = cs;
        if (k + 1 < ny) A[q * width + bw + w] = cn;
        b[q] = U[(long)k * nx + i];
      }
    band_lu(A, n, bw);
    memcpy(x, b, sizeof(double) * n);
    band_solve(A, n, bw, x);
    /* refinement: residual of the original rows (rebuilt by dd2_row) in long double */
    double* d = (double*)malloc(sizeof(double) * n);
    for (int k = 0; k < ny; k++)
      for (int i = i0; i < i1; i++) {
        const long q = (long)k * w + (i - i0);
        double cw, ce, cs, cn;
        const double dg = dd2_row(p, r, tau, i, k, &cw, &ce, &cs, &cn);
        long double acc = (long double)b[q] - (long double)dg * x[q];
        if (i > i0) acc -= (long double)cw * x[q - 1];
        if (i + 1 < i1) acc -= (long double)ce * x[q + 1];
        if (k > 0) acc -= (long double)cs * x[q - w];
        if (k + 1 < ny) acc -= (long double)cn * x[q + w];
        d[q] = (double)acc;
      }
    band_solve(A, n, bw, d);
    for (int k = 0; k < ny; k++)
      for (int i = i0; i < i1; i++) {
        const long q = (long)k * w + (i - i0);
        U[(long)k * nx + i] = x[q] + d[q];
      }
    free(A);
    free(b);
    free(x);
    free(d);
    i0 = i1;
  }
}

/* A_j U for the 2D domain-decomposition split (the operator of dd2_row). */
static void dd2_apply(const or_problem* p, int j, const double* U, double* out) {
  const int nx = p->nx, ny = p->ny;
  const double* r = p->rho + (long)j * (2 * nx + 1);
  for (int k = 0; k < ny; k++)
    for (int i = 0; i < nx; i++) {
      double cw, ce, cs, cn;
      const double d = dd2_row(p, r, 1.0, i, k, &cw, &ce, &cs, &cn) - 1.0;
      const double u = U[(long)k * nx + i];
      const double uw = (i > 0) ? U[(long)k * nx + i - 1] : 0.0;
      const double ue = (i < nx - 1) ? U[(long)k * nx + i + 1] : 0.0;
      const double us = (k > 0) ? U[(long)(k - 1) * nx + i] : 0.0;
      const double un = (k < ny - 1) ? U[(long)(k + 1) * nx + i] : 0.0;
      /* with tau = 1 the couplings are minus the flux weights */
      out[(long)k * nx + i] = -(cw * uw + ce * ue + cs * us + cn * un) - d * u;
    }
}

/* One implicit substep (I - tau*A_j) V = U along every line of the split
 * term j, in place. j = 0: x-lines (dimensional) or colour 0 (domain
 * decomposition). */
static void implicit_substep(const or_problem* p, int j, double tau, double* U) {
  const int nx = p->nx, ny = p->ny;
  if (p->split == 0) {
    const int M = p->dim;
    const double react = p->c / M; /* the reaction is shared equally, section 2.1 */
    if (j == 0) {
      line_ws w = ws_alloc(nx);
      for (int row = 0; row < ny; row++) {
        assemble_line(nx, p->ax + (long)row * (nx + 1), 1, hx_of(p), tau, react, &w);
        thomas(nx, w.lo, w.di, w.up, U + (long)row * nx, w.cp);
      }
      ws_free(&w);
    } else {
      line_ws w = ws_alloc(ny);
      for (int col = 0; col < nx; col++) {
        assemble_line(ny, p->ay + col, nx, hy_of(p), tau, react, &w);
        for (int r = 0; r < ny; r++) w.rhs[r] = U[(long)r * nx + col];
        thomas(ny, w.lo, w.di, w.up, w.rhs, w.cp);
        for (int r = 0; r < ny; r++) U[(long)r * nx + col] = w.rhs[r];
      }
      ws_free(&w);
    }
  } else if (p->dim == 2) {
    dd2_substep(p, j, tau, U);
  } else {
    /* Domain decomposition (1D): the operator of colour j uses the face
     * coefficient rho_j * a. Where rho_j vanishes on both faces of a node the
     * row is the identity, so the whole-line system is block diagonal with one
     * block per connected component plus identity rows; solving it as one
     * tridiagonal system is the definition of the substep. */
    double* wface = (double*)malloc(sizeof(double) * (nx + 1));
    for (int f = 0; f <= nx; f++) wface[f] = p->rho[(long)j * (nx + 1) + f] * p->ax[f];
    line_ws w = ws_alloc(nx);
    assemble_line(nx, wface, 1, hx_of(p), tau, 0.0, &w);
    thomas(nx, w.lo, w.di, w.up, U, w.cp);
    ws_free(&w);
    free(wface);
  }
}

/* Stencil application of one split operator along the lines of term j:
 * (A_j U)_i = [w_{i+1}(U_{i+1}-U_i) - w_i(U_i-U_{i-1})]/h^2 - react*U_i
 * with U = 0 outside the grid. */
static void apply_line(int n, const double* face, long face_stride, double h, double react,
                       const double* u, long us, double* out, long os, int accumulate) {
  for (int i = 0; i < n; i++) {
    double ui = u[(long)i * us];
    double ul = (i > 0) ? u[(long)(i - 1) * us] : 0.0;
    double ur = (i < n - 1) ? u[(long)(i + 1) * us] : 0.0;
    double aw = face[(long)i * face_stride];
    double ae = face[(long)(i + 1) * face_stride];
    double v = (ae * (ur - ui) - aw * (ui - ul)) / (h * h) - react * ui;
    if (accumulate)
      out[(long)i * os] += v;
    else
      out[(long)i * os] = v;
  }
}

void or_apply_Aj(const or_problem* p, int j, const double* U, double* out) {
  const int nx = p->nx, ny = p->ny;
  if (p->split == 0) {
    const double react = p->c / p->dim;
    if (j == 0) {
      for (int row = 0; row < ny; row++)
        apply_line(nx, p->ax + (long)row * (nx + 1), 1, hx_of(p), react, U + (long)row * nx, 1,
                   out + (long)row * nx, 1, 0);
    } else {
      for (int col = 0; col < nx; col++)
        apply_line(ny, p->ay + col, nx, hy_of(p), react, U + col, nx, out + col, nx, 0);
    }
  } else if (p->dim == 2) {
    dd2_apply(p, j, U, out);
  } else {
    double* wface = (double*)malloc(sizeof(double) * (nx + 1));
    for (int f = 0; f <= nx; f++) wface[f] = p->rho[(long)j * (nx + 1) + f] * p->ax[f];
    apply_line(nx, wface, 1, hx_of(p), 0.0, U, 1, out, 1, 0);
    free(wface);
  }
}

void or_apply_A(const or_problem* p, const double* U, double* out) {
  const int npts = npts_of(p);
  double* tmp = (double*)malloc(sizeof(double) * npts);
  memset(out, 0, sizeof(double) * npts);
  for (int j = 0; j < n_terms(p); j++) {
    or_apply_Aj(p, j, U, tmp);
    for (int k = 0; k < npts; k++) out[k] += tmp[k];
  }
  free(tmp);
}

void or_faces_from_theta_1d(int nx, const double* theta, double* ax) {
  for (int f = 0; f <= nx; f++) ax[f] = 0.5 * (exp(theta[f]) + exp(theta[f + 1]));
}

void or_faces_from_theta(int nx, int ny, const double* theta, double* ax, double* ay) {
  const int W = nx + 2; /* theta row stride, boundary nodes included */
  for (int j = 0; j < ny; j++)
    for (int f = 0; f <= nx; f++) {
      /* face f of interior row j joins extended nodes (f, j+1) and (f+1, j+1) */
      double tp = theta[(long)(j + 1) * W + f];
      double tq = theta[(long)(j + 1) * W + f + 1];
      ax[(long)j * (nx + 1) + f] = 0.5 * (exp(tp) + exp(tq));
    }
  if (ay)
    for (int g = 0; g <= ny; g++)
      for (int i = 0; i < nx; i++) {
        double tp = theta[(long)g * W + i + 1];
        double tq = theta[(long)(g + 1) * W + i + 1];
        ay[(long)g * nx + i] = 0.5 * (exp(tp) + exp(tq));
      }
}

/* FIE, eq. FIE_method: (I - tau A_1) U_1 = U_n + tau F_{n+1},
 * (I - tau A_j) U_j = U_{j-1}, U_{n+1} = U_M. */
void or_fie_step(const or_problem* p, double tau, const double* F, double* U) {
  if (F)
    for (int k = 0; k < npts_of(p); k++) U[k] = U[k] + tau * F[k];
  for (int j = 0; j < n_terms(p); j++) implicit_substep(p, j, tau, U);
}

/* Douglas-Rachford, eq. DR_method:
 * U_0 = (I + tau A) U_n + tau F_{n+1}, (I - tau A_j) U_j = U_{j-1} - tau A_j U_n. */
void or_dr_step(const or_problem* p, double tau, const double* F, double* U) {
  const int npts = npts_of(p);
  double* Un = (double*)malloc(sizeof(double) * npts);
  double* AU = (double*)malloc(sizeof(double) * npts);
  double* V = (double*)malloc(sizeof(double) * npts);
  memcpy(Un, U, sizeof(double) * npts);
  or_apply_A(p, Un, AU);
  for (int k = 0; k < npts; k++) V[k] = Un[k] + tau * AU[k];
  if (F)
    for (int k = 0; k < npts; k++) V[k] = V[k] + tau * F[k];
  for (int j = 0; j < n_terms(p); j++) {
    or_apply_Aj(p, j, Un, AU);
    for (int k = 0; k < npts; k++) V[k] = V[k] - tau * AU[k];
    implicit_substep(p, j, tau, V);
  }
  memcpy(U, V, sizeof(double) * npts);
  free(Un);
  free(AU);
  free(V);
}

/* Source F at one time level: F = sum_m table[m*stride + idx] S_m. Returns
 * NULL (F = 0) when the problem has no source terms. */
static double* source_at(const or_problem* p, const double* table, long stride, long idx) {
  if (p->n_forcing <= 0) return NULL;
  const long npts = npts_of(p);
  double* F = (double*)calloc(npts, sizeof(double));
  for (int m = 0; m < p->n_forcing; m++) {
    const double g = table[m * stride + idx];
    for (long q = 0; q < npts; q++) F[q] = F[q] + g * p->fS[m * npts + q];
  }
  return F;
}

/* Fine propagator: s steps of the fine method at dt = DT/s over coarse
 * interval n (section 3). */
void or_fine(const or_problem* p, int n, double* U) {
  const double DT = p->T / p->n_slices;
  const double dt = DT / p->fine_steps;
  const long stride = (long)p->n_slices * p->fine_steps;
  for (int t = 0; t < p->fine_steps; t++) {
    double* F = source_at(p, p->fg_fine, stride, (long)n * p->fine_steps + t);
    if (p->fine_method == 1)
      or_dr_step(p, dt, F, U);
    else
      or_fie_step(p, dt, F, U);
    free(F);
  }
}

/* Coarse propagator: FIE (L-stable, section 4) with coarse_steps steps over
 * coarse interval n. */
void or_coarse(const or_problem* p, int n, double* U) {
  const double DT = p->T / p->n_slices;
  const double tau = DT / p->coarse_steps;
  const long stride = (long)p->n_slices * p->coarse_steps;
  for (int t = 0; t < p->coarse_steps; t++) {
    double* F = source_at(p, p->fg_coarse, stride, (long)n * p->coarse_steps + t);
    or_fie_step(p, tau, F, U);
    free(F);
  }
}

void or_fine_batch(const or_problem* p, int n, const double* U_in, double* F_out) {
  const long npts = npts_of(p);
  for (int k = 0; k < n; k++) {
    memcpy(F_out + k * npts, U_in + k * npts, sizeof(double) * npts);
    or_fine(p, k, F_out + k * npts);
  }
}

void or_sequential_fine(const or_problem* p, const double* u0, double* U) {
  const long npts = npts_of(p);
  memcpy(U, u0, sizeof(double) * npts);
  for (int n = 0; n < p->n_slices; n++) {
    memcpy(U + (n + 1) * npts, U + n * npts, sizeof(double) * npts);
    or_fine(p, n, U + (n + 1) * npts);
  }
}

double or_coarse_sweep(const or_problem* p, const double* F, double* G_old, double* U) {
  const long npts = npts_of(p);
  const int N = p->n_slices;
  double* g = (double*)malloc(sizeof(double) * npts);
  double inc = 0.0;
  for (int n = 0; n < N; n++) {
    memcpy(g, U + n * npts, sizeof(double) * npts);
    or_coarse(p, n, g); /* g = G(U^{k+1}_n) */
    double* Unext = U + (n + 1) * npts;
    double* Gn = G_old + n * npts;
    for (long q = 0; q < npts; q++) {
      double v;
      if (F)
        v = F[n * npts + q] + (g[q] - Gn[q]);
      else
        v = g[q];
      double d = fabs(v - Unext[q]);
      if (F && d > inc) inc = d;
      Unext[q] = v;
      Gn[q] = g[q];
    }
  }
  free(g);
  return inc;
}

int or_parareal(const or_problem* p, const double* u0, int k_max, double tol, double* U,
                double* inc_hist) {
  const long npts = npts_of(p);
  const int N = p->n_slices;
  double* G_old = (double*)malloc(sizeof(double) * N * npts);
  double* F = (double*)malloc(sizeof(double) * N * npts);
  memcpy(U, u0, sizeof(double) * npts);
  or_coarse_sweep(p, NULL, G_old, U); /* U^0_{n+1} = G(U^0_n) */
  int k = 0;
  while (k < k_max) {
    or_fine_batch(p, N, U, F); /* F_n = F^s(U^k_n) for n = 0..N-1 */
    double inc = or_coarse_sweep(p, F, G_old, U);
    if (inc_hist) inc_hist[k] = inc;
    k++;
    if (inc < tol) break;
  }
  free(G_old);
  free(F);
  return k;
}

/* Adjoint of the fine map.
 * One FIE step is W = Bx^{-1} U, V = By^{-1} W with Bx = I - tau A_x and
 * By = I - tau A_y, both symmetric. For L = <lambda, V>:
 *   mu = By^{-1} lambda,   nu = Bx^{-1} mu,   dL/dU = nu;
 * and since dBy/da_f = -tau dA_y/da_f, dL/da_f = tau mu^T (dA_y/da_f) V, i.e.
 *   dL/da_f = -(tau/h^2) (mu_q - mu_p)(V_q - V_p) for a y-face f = (p, q),
 * with mu = V = 0 on boundary nodes (x-faces likewise with nu and W).
 * Steps are reversed one by one; the forward states of each slice are
 * recomputed from the slice's starting state. */
static void face_grad_x(int nx, int ny, double coef, const double* mu, const double* V,
                        double* gax) {
  for (int j = 0; j < ny; j++)
    for (int f = 0; f <= nx; f++) {
      double mp = (f > 0) ? mu[(long)j * nx + f - 1] : 0.0;
      double mq = (f < nx) ? mu[(long)j * nx + f] : 0.0;
      double vp = (f > 0) ? V[(long)j * nx + f - 1] : 0.0;
      double vq = (f < nx) ? V[(long)j * nx + f] : 0.0;
      gax[(long)j * (nx + 1) + f] += -coef * (mq - mp) * (vq - vp);
    }
}

static void face_grad_y(int nx, int ny, double coef, const double* mu, const double* V,
                        double* gay) {
  for (int g = 0; g <= ny; g++)
    for (int i = 0; i < nx; i++) {
      double mp = (g > 0) ? mu[(long)(g - 1) * nx + i] : 0.0;
      double mq = (g < ny) ? mu[(long)g * nx + i] : 0.0;
      double vp = (g > 0) ? V[(long)(g - 1) * nx + i] : 0.0;
      double vq = (g < ny) ? V[(long)g * nx + i] : 0.0;
      gay[(long)g * nx + i] += -coef * (mq - mp) * (vq - vp);
    }
}

void or_adjoint(const or_problem* p, const double* u0, const double* lambda_T, double* grad_u0,
                double* grad_ax, double* grad_ay) {
  const int nx = p->nx, ny = p->ny, N = p->n_slices, s = p->fine_steps;
  const long npts = npts_of(p);
  const double dt = p->T / N / s;
  double* ckpt = (double*)malloc(sizeof(double) * (N + 1) * npts);
  double* Wst = (double*)malloc(sizeof(double) * s * npts); /* after x substep */
  double* Vst = (double*)malloc(sizeof(double) * s * npts); /* after y substep */
  double* lam = (double*)malloc(sizeof(double) * npts);
  or_sequential_fine(p, u0, ckpt);
  memset(grad_ax, 0, sizeof(double) * ny * (nx + 1));
  if (p->dim == 2) memset(grad_ay, 0, sizeof(double) * (ny + 1) * nx);
  memcpy(lam, lambda_T, sizeof(double) * npts);
  for (int n = N - 1; n >= 0; n--) {
    double* cur = (double*)malloc(sizeof(double) * npts);
    memcpy(cur, ckpt + (long)n * npts, sizeof(double) * npts);
    for (int t = 0; t < s; t++) {
      /* the source enters the x substep's right-hand side; the face gradients
       * below only need the post-substep states */
      double* F = source_at(p, p->fg_fine, (long)N * s, (long)n * s + t);
      if (F)
        for (long q = 0; q < npts; q++) cur[q] = cur[q] + dt * F[q];
      free(F);
      implicit_substep(p, 0, dt, cur);
      memcpy(Wst + (long)t * npts, cur, sizeof(double) * npts);
      if (p->dim == 2) implicit_substep(p, 1, dt, cur);
      memcpy(Vst + (long)t * npts, cur, sizeof(double) * npts);
    }
    free(cur);
    for (int t = s - 1; t >= 0; t--) {
      if (p->dim == 2) {
        implicit_substep(p, 1, dt, lam); /* lam <- mu */
        face_grad_y(nx, ny, dt / (hy_of(p) * hy_of(p)), lam, Vst + (long)t * npts, grad_ay);
      }
      implicit_substep(p, 0, dt, lam); /* lam <- nu */
      face_grad_x(nx, ny, dt / (hx_of(p) * hx_of(p)), lam, Wst + (long)t * npts, grad_ax);
    }
  }
  memcpy(grad_u0, lam, sizeof(double) * npts);
  free(ckpt);
  free(Wst);
  free(Vst);
  free(lam);
}

void or_theta_grad(int nx, int ny, const double* theta, const double* grad_ax,
                   const double* grad_ay, double* grad_theta) {
  const int W = nx + 2;
  memset(grad_theta, 0, sizeof(double) * (long)(nx + 2) * (ny + 2));
  for (int j = 0; j < ny; j++)
    for (int f = 0; f <= nx; f++) {
      double gf = grad_ax[(long)j * (nx + 1) + f];
      long p0 = (long)(j + 1) * W + f, q0 = p0 + 1;
      grad_theta[p0] += 0.5 * exp(theta[p0]) * gf;
      grad_theta[q0] += 0.5 * exp(theta[q0]) * gf;
    }
  if (grad_ay)
    for (int g = 0; g <= ny; g++)
      for (int i = 0; i < nx; i++) {
        double gf = grad_ay[(long)g * nx + i];
        long p0 = (long)g * W + i + 1, q0 = p0 + W;
        grad_theta[p0] += 0.5 * exp(theta[p0]) * gf;
        grad_theta[q0] += 0.5 * exp(theta[q0]) * gf;
      }
}
