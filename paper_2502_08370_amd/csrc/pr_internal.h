// Internal declarations shared by the host runtime and the HIP kernels of the
// parareal-with-splitting library. Not part of the public ABI (include/pr.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace prk {

// Device-side description of one dimensional-splitting instance.
//
// Fine workspace layout ("interleaved"): the N slices of an instance are
// grouped in B blocks of L consecutive slices (L a power of two <= 64,
// padding slices are zero). Block b holds Z[b][j][i][l]: for each grid node
// the L slice values are contiguous, so a wave whose lanes walk (line, slice)
// reads and writes whole 8*L-byte segments at every step of a line solve, in
// both sweep directions, and every lane of a line shares the same
// factorisation entries.
//
// Line systems (I - tau A_dir) are factorised once per tau (LU without
// pivoting, diagonally dominant M-matrix): with w_f = tau a_f / h^2,
//   forward   y_p = d_p + e_p y_{p-1}
//   backward  x_p = r_p y_p + g_p x_{p+1}
// e_p = w_p / u_{p-1}, r_p = 1 / u_p, g_p = w_{p+1} / u_p, u the LU pivots.
// The fine sweeps split each line into chunks of M positions and leave the
// back substitution of every chunk uncoupled (x_{chunk end + 1} taken as 0);
// the exact result is z_p + phi_p * sigma_k with phi_p = prod_{t=p..end} g_t
// and sigma_k the true value just past chunk k. The consumer of a sweep's
// output (the next sweep or the final transpose) adds phi_p * sigma_k when it
// loads, so each sweep moves every value through HBM exactly once.
struct DimInst {
  int nx, ny;        // interior nodes
  int N;             // slices
  int L, B;          // lanes per slice block, number of slice blocks
  int M;             // chunk length of the fine sweeps
  int Px, Py;        // chunks per x-line (ceil(nx/M)), per y-line (ceil(ny/M))
  // Twisted fine factorisation: x-line positions from chunk twx on (y-lines: twy)
  // hold the UL factors of the line's bottom part (r_p = 1 / v_p, g_p = w_p / v_p,
  // v the pivots eliminated from the line end), the positions before them the
  // LU factors of the top part; twx = Px (twy = Py) when the lines are not twisted.
  int twx, twy;
  int steps;         // fine steps per slice; grouped sweeps skip instances past it
  long slab;         // doubles per slice block of Z: ny*nx*L
  double* Z;         // [B][ny][nx][L]
  long zout;         // fine sweeps store at Z + zout (0: in place)
  double* sigX;      // [B][Px][ny][L]  chunk carries of the x sweep
  double* sigY;      // [B][Py][nx][L]  chunk carries of the y sweep
  // fine factorisations, line-major: x-line j entry (j*nx + i), y-line i entry (i*ny + j)
  const double* fxR; const double* fxG;
  const double* fyR; const double* fyG;
  // the same as (r, g) pairs, [line][pos][2], for one 16-byte load per position
  const double* fxRG; const double* fyRG;
  // phi of the fine sweeps, stored where their consumer reads them:
  //   fxPhiC[i*ny + j]: x-line j, position i (read by y-lines)
  //   fyPhiC[j*nx + i]: y-line i, position j (read by x-lines and the final transpose)
  //   fxPhiS[j*Px + k], fyPhiS[i*Py + k]: phi at the first position of chunk k
  const double* fxPhiC; const double* fyPhiC;
  const double* fxPhiS; const double* fyPhiS;
  // Partitioned fine sweeps (few slices, see launch_part_sweep): positions per
  // part of an x-line / y-line (0: not used); their own slice blocks of Lp
  // slices (Bp blocks, the last one possibly shorter; no padding) laid out as
  // Z[b][j][i][l] with slabp = nx*ny*Lp doubles per block; and the plain LU of
  // the fine line systems as (r, g) pairs, [line][pos][2], whatever form the
  // other sweeps use
  int plx, ply;
  int Lp, Bp;
  long slabp;
  const double* pxRG; const double* pyRG;
  // Lane-blocked factor copies for the one-wave-per-line solvers (coarse
  // propagator, sequential fine solve, adjoint): line l, segment s, position
  // p = s*64*K + lane*K + c at [l][s][c][lane], zero past the line end; K = Kx,
  // Sx segments for x-lines, Ky, Sy for y-lines (S > 1 only when K = 16).
  int Kx, Ky, Sx, Sy;
  const double* cxRb; const double* cxGb; const double* cyRb; const double* cyGb;
  const double* fxRb; const double* fxGb; const double* fyRb; const double* fyGb;
  double* tmp;       // one-state scratch of the coarse sweep
  unsigned long long* incp;  // per-block increment maxima of a coarse sweep
  int n_incp;                // their count
  // batch bookkeeping
  int idx;           // instance index in the handle
  int cs;            // coarse steps per coarse propagation
  long npts;         // nx*ny
  long off_slices, off_states;  // offsets of the instance in packed buffers
  const int* active; // per-instance flags (0: converged, skipped by every kernel)
  // Douglas-Rachford fine propagator (eq. DR_method): S = dt A_y U of the step's
  // input, stored like Z. The x sweep adds it on load (and writes back S with
  // its pending correction applied), the y sweep subtracts it; since the y
  // stage solves (I - dt A_y) U' = Y, the next step's S = dt A_y U' = U' - Y is
  // formed by the y sweep itself (stored with U''s pending chunk correction)
  int dr;
  double* drS;       // [B][ny][nx][L]
  const double* ay;  // y-face coefficients [(ny+1)][nx]
  double dr_coef;    // dt / h_y^2
  double dr_react;   // dt * c / 2
  // source F(t) = sum_m g_m(t) S_m of eq. FIE_method / eq. DR_method; tau F at
  // the step's end time enters its first stage (the x substep, the x sweep's load)
  int nforce;        // 0: no source
  const double* fS;  // [kMaxForcing][npts] (unused terms zero)
  const double* fgf; // [kMaxForcing][N * steps]: dt * g_m at the fine step ends
  const double* fgc; // [kMaxForcing][N * cs]: (DT / cs) * g_m at the coarse step ends
};

constexpr int kMaxForcing = 2;
constexpr int kDRChunk = 16;  // chunk length of the Douglas-Rachford sweeps

// Work item of a batched coarse launch: instance and line block.
struct LineItem {
  int inst, block;
};

// Work item of a grouped fine-sweep launch: instance, slice block, line group.
struct WorkItem {
  int inst, b, group, pad;
};

// Factorisation of one direction of one instance at one tau.
struct FactorJob {
  const double* face;  // face coefficients of this direction
  int n_lines, n_pos;  // lines and positions per line
  long face_line_stride, face_pos_stride;  // in doubles
  double tau_over_h2;  // tau / h^2
  double react;        // tau * c / M added to the diagonal
  double* E; double* R; double* G;  // outputs (E may be NULL)
  int pos_major;       // 0: [line][pos], 1: [pos][line]
  int pad;
};

// ---------------------------------------------------------------------------
// Domain-decomposition splitting in 1D (section 2.1: L_k u = (rho_k a u_x)_x,
// partition of unity rho_k). The substep of colour k solves (I - tau A_k) on
// each connected component of colour k (a run of faces with rho_k > 0) and
// leaves every other node unchanged. Components are long, so each is cut into
// segments of kDDSeg nodes: phase 1 solves every segment with zero carries in
// both directions using the component's LU factors, phase 2 resolves the
// carries across the segments of each component, phase 3 adds them:
//   x_i = z_i + chi_i Yin + phi_i Xin
// with Yin the forward-elimination value just before the segment and Xin the
// solution just after it; chi_i is the back-substituted product of forward
// multipliers and phi_i the product of back-substitution multipliers.
constexpr int kDDSeg = 32;

struct DDSeg {
  int lo, len;    // first node, node count (<= kDDSeg)
  int comp;       // component index
  int colour;
};

// One set of factors (one tau) for all colours, indexed [colour][node].
struct DDFactors {
  const double* R; const double* G;  // e_i = G[i-1] (see k_dd_factorize)
  const double* CHI; const double* PHI;
  const double* PSIE;  // per segment: product of e over the segment
  const double* CHIA;  // per segment: chi at its first node
  const double* PHIA;  // per segment: phi at its first node
  // Deferred corrections (fine set only, else NULL): chi and phi of the
  // correction a node carries when colour k loads it, [colour][node], at the
  // first step (PC0, PP0: same-step sources only) and later (PC1, PP1); and of
  // the correction it carries after the last substep (FC, FP: [node]).
  const double* PC0; const double* PP0; const double* PC1; const double* PP1;
  const double* FC; const double* FP;
  // Per segment t of its run (slice-independent parts of the carries, see
  // DDInst): SA = product of PSIE over the run's segments before t; the X after
  // segment t is SC RX + SD RY + (its slice part).
  const double* SA; const double* SC; const double* SD;
};

// The carries are resolved over runs of kDDRun consecutive segments of one
// component: each run is summarised by the affine maps that give its last Y and
// its first X from the Y before it and the X after it (2a), one wave scan per
// component and slice chains the runs (2b), and each run then re-derives the
// carries of its segments (2c).
constexpr int kDDRun = 16;

struct DDRun {
  int seg0, len;  // first segment (index into segs), segment count (<= kDDRun)
};

// Everything the slice-interleaved segment solves of one run look up, in one
// record (one level of loads before the values): per segment t of the run its
// node range and the pending-correction source (first step, later steps; -1:
// none) with that source's run.
struct DDRunRec {
  int seg0, len;
  int lo[kDDRun], cnt[kDDRun];
  int src[2][kDDRun], srun[2][kDDRun];
};

struct DDInst {
  int n, N, L, B;       // nodes, slices, lanes per slice block, slice blocks
  int n_colors, n_segs;  // colours, segments of all colours
  long slab;            // doubles per slice block of Z: n*L
  double* Z;            // [B][n][L] (fine) or the state itself (L = 1)
  const DDSeg* segs;    // [n_segs], colour-major
  // per (segment, slice): [B][n_segs][L]; the carries of the slice-interleaved
  // workspace after its last substep (k_dd_final_carries)
  double* Yin; double* Xin;
  // The carries of segment t of run r are formed where they are used,
  // Yin = SA_t RY_r + Yp_t and Xin = SC_t RX_r + SD_t RY_r + Xp_t, from the run's
  // carries and the slice parts Yp, Xp ([B][n_segs][L]) that the run maps leave.
  double* Yp; double* Xp;
  const int* seg_run;   // [n_segs]: the run that holds the segment
  int n_runs;           // runs of all colours
  const DDRun* runs;    // [n_runs], colour-major, runs of a component contiguous
  // per (run, slice): [B][n_runs][L]. Run maps: Y_last = P Y_before + Q,
  // X_first = U X_after + V Y_before + W; run carries RY = Y_before, RX = X_after.
  double* RP; double* RQ; double* RU; double* RV; double* RW; double* RY; double* RX;
  // Deferred corrections (fine substeps): a segment's phase-1 output is left as
  // z; the exact value z + chi Yin + phi Xin is formed by the next load of the
  // node. Per segment: the segment whose correction its nodes carry when it is
  // loaded at the first step (seg_src0: an earlier colour of the same step, or
  // -1) and at later steps (seg_src1: the same, else the previous step's last
  // colour covering it); per node: the segment whose correction it carries
  // after the last substep (fin_seg).
  const int* seg_src0; const int* seg_src1; const int* fin_seg;
  const DDRunRec* run_recs;  // [n_runs]
};

// Phase 1, one workgroup per run [run_begin, run_begin + run_count) of the
// colour, which also chains the run's segments (the slice parts Yp, Xp and the
// run maps of phase 2). Single state (L = 1): zero-carry segment solves of an
// input that carries no correction (phase 3 corrects in place). Slice-
// interleaved workspace (L >= 8): the pending correction of the previous
// substeps is applied on load (stale_ok: the previous step's corrections
// exist) and this one is left pending. seg_begin, seg_count: the colour's
// segments (unused by the kernels; kept for the caller's bookkeeping).
hipError_t launch_dd_local(const DDInst* d, const DDInst& h, const DDFactors& f, int colour,
                           int seg_begin, int seg_count, int run_begin, int run_count,
                           bool stale_ok, hipStream_t s);
// Interleaved Z with the pending corrections of the last substeps -> natural
// F[slice][node].
hipError_t launch_dd_from_interleaved(const DDInst* d, const DDInst& h, const DDFactors& f,
                                      double* F, hipStream_t s);
// Runs [run_begin, run_begin + run_count) of one colour; comp_run_first /
// comp_run_count (device, n_comps entries) list each component's runs. The
// slice-interleaved workspace only needs the scan over runs (its run maps come
// from launch_dd_local).
hipError_t launch_dd_carries(const DDInst* d, const DDInst& h, const DDFactors& f, int run_begin,
                             int run_count, const int* comp_run_first, const int* comp_run_count,
                             int n_comps, hipStream_t s);
// Phase 3 of the single state (L = 1).
hipError_t launch_dd_correct(const DDInst* d, const DDInst& h, const DDFactors& f, int colour,
                             int seg_begin, int seg_count, hipStream_t s);
// SA, SC, SD of every run's segments (written through the given pointers).
hipError_t launch_dd_runfactors(const DDInst* d, const DDInst& h, const DDFactors& f, double* SA,
                                double* SC, double* SD, hipStream_t s);
// Set-up: component LU (one thread per component) and segment factors.
hipError_t launch_dd_faces(const double* rho, const double* a, int n, int n_colors, double* w,
                           hipStream_t s);
hipError_t launch_dd_factorize(const double* w, int n, const int* comp_lo, const int* comp_hi,
                               const int* comp_colour, int n_comps, double tau_over_h2, double* R,
                               double* G, hipStream_t s);
hipError_t launch_dd_segfactors(const DDSeg* segs, const int* seg_colour, int n_segs, int n,
                                const double* R, const double* G, double* CHI,
                                double* PHI, double* PSIE, double* CHIA, double* PHIA,
                                hipStream_t s);
// Pending-correction factors of the deferred fine substeps (PC0, PP0, PC1,
// PP1, FC, FP of f, written through the given non-const pointers).
hipError_t launch_dd_pending(const DDInst* d, const DDInst& h, const DDFactors& f, double* PC0,
                             double* PP0, double* PC1, double* PP1, double* FC, double* FP,
                             hipStream_t s);
// Parareal correction over whole states: U_next = F + (g - G_old), G_old = g,
// increment (mode 1), or U_next = G_old = g (mode 2). The increment goes to
// partial[0 .. update_blocks(n)) as per-block maxima (see launch_inc_reduce).
int update_blocks(size_t n);
hipError_t launch_update(const double* g, const double* F, double* G_old, double* U_next,
                         size_t n, int mode, unsigned long long* partial, hipStream_t s);

// ---------------------------------------------------------------------------
// Domain-decomposition splitting in 2D with vertical strips (section 2.1, the
// subdomains of Fig. fig:domaindecomposition). The partition of unity depends
// on x only and is sampled on the half grid of x (x-faces and node columns).
// The substep of colour k solves (I - tau A_k) on each strip of colour k (a
// maximal run of columns where rho_k is nonzero on the node or an x-face) and
// leaves every other column unchanged. A strip of w columns is a 5-point
// system, block tridiagonal in y with w x w blocks: D_r (tridiagonal in x) on
// the diagonal and the diagonal y couplings b_r (to row r-1) and c_r (to row
// r+1) beside it. It is solved exactly by block cyclic reduction in y: at level
// l the rows alive are r = 2^l (a+1) - 1; even a are eliminated, odd a kept,
// neighbours at distance 2^l. Per eliminated row the solve forms y = D^-1 r;
// per kept row r -= B y_- + C y_+; going back down, x = y - M2 x_- - M3 x_+
// with M2 = D^-1 B, M3 = D^-1 C. At level 0, where D is tridiagonal and B, C
// are diagonal, y = D^-1 r and the back substitution x = y - D^-1 (b x_- +
// c x_+) are Thomas solves with the LU of D (multipliers, reciprocal pivots and
// back factors, 3 W doubles per row, "tri" arrays) and the kept-row update is
// elementwise. The blocks of levels >= 1 are dense (fill-in); they are
// precomputed per tau ("factor pool") in the operand layout of the FP64 MFMA
// (16x16x4): element (o, k) of a matrix padded to W (a multiple of 16) sits at
// dd2_frag(W, o, k). The solve streams each matrix once per substep for all
// slices, which sit contiguously at every grid node ("slice-minor" layout
// Zs[node][b], b < Npad).
constexpr int kDD2MaxW = 1024;  // widest padded strip
constexpr int kDD2WholeRowTiles = 2;  // row tiles per wave in the whole-row solve launches
constexpr int kDD2SplitTiles = 2;     // most row tiles per unit in the other launches

__host__ __device__ inline long dd2_frag(int W, int o, int k) {
  return ((long)(k >> 2) * (W >> 4) + (o >> 4)) * 64 + (k & 3) * 16 + (o & 15);
}

// One wave's share of a solve launch: rows [16 mb0, 16 (mb0 + nmb)) of the
// output of block row `row` of the strip at columns [col0, col0 + w).
struct DD2Unit {
  int col0, w, W, row;
  int mb0, nmb, rowm, rowp;  // neighbour block rows (-1: none)
  long A0, A1, A2;           // matrix offsets in the factor pool (per mode)
  long bc;                   // offset of the row's coupling vectors b, c
};

// Row of level 0: a kept row (elementwise update r -= b y_- + c y_+) or an
// eliminated row (Thomas solves with its LU at tri: multipliers m, reciprocal
// pivots ip and back factors g, W doubles each).
struct DD2Row {
  int col0, w, W, row, rowm, rowp;
  long bc;   // b_row at bc, c_row at bc + W
  long tri;  // eliminated rows: offset in the tri arrays (-1 for kept rows)
};

// Strip geometry and coefficients for the set-up kernels.
struct DD2Geo {
  const double* ax;   // x-faces [ny][nx+1]
  const double* ay;   // y-faces [ny+1][nx]
  const double* rho;  // this colour's half-grid weights [2nx+1]
  int nx, ny;
  int col0, w, W, pad;
  double tx, ty;      // tau / h_x^2, tau / h_y^2
  double tc;          // tau * c
};

// Set-up jobs: C = base + sgn * A B over W x W blocks (base NULL: 0), and
// dense-to-pool copies.
struct DD2Gemm {
  const double* A; const double* B; const double* base; double* C;
  int lda, ldb, ldbase, ldc;
  double sgn;
};
struct DD2Copy {
  const double* src; double* dst;
  int ld, pad;
};

// Solve phases: MFMA phases over units (levels >= 1), then the row phases of
// level 0.
enum { DD2_APPLY = 0, DD2_KUP = 1, DD2_BACK = 2, DD2_KUP0 = 3, DD2_TRI_APPLY = 4, DD2_TRI_BACK = 5 };

// ---- launchers (pr_kernels_dd2.hip) ----
// Coupling vectors of every block row: bc[r][0][o] = b_r, bc[r][1][o] = c_r
// (zero past w, b_0 = c_{ny-1} = 0).
hipError_t launch_dd2_bc(const DD2Geo& g, double* bc, hipStream_t s);
// Inverses of the level-0 blocks (tridiagonal) of the eliminated rows r = 2m,
// m < n, into columns [W, 2W) of the matrix at aug + m * mstride (row stride 2W),
// and their LU (m, ip, g; 3 W doubles per row) at tri + 3 W m.
hipError_t launch_dd2_tri_inv(const DD2Geo& g, int n, double* aug, long mstride, double* tri,
                              hipStream_t s);
// Gauss-Jordan on n augmented matrices [D | R] (W rows, LD columns): D -> I, R -> D^-1 R.
hipError_t launch_dd2_gj(double* aug, long mstride, int n, int W, int LD, hipStream_t s);
// Level-1 blocks of the level-0 kept rows r = 2a + 1 (a < ny / 2) from the
// level-0 inverses (columns [W, 2W) of aug0): D, B, C with leading dimension W.
hipError_t launch_dd2_scale0(const DD2Geo& g, const double* bc, const double* aug0, long mstride,
                             double* Dn, double* Bn, double* Cn, hipStream_t s);
// [D_a | I | B_a | C_a] (row stride 4W) for the eliminated rows a = 2e, e < nE.
hipError_t launch_dd2_aug(const double* D, const double* B, const double* C, int nE, int W,
                          double* aug, hipStream_t s);
hipError_t launch_dd2_gemm(const DD2Gemm* jobs, int n, int W, hipStream_t s);
hipError_t launch_dd2_store(const DD2Copy* jobs, int n, int W, hipStream_t s);
// One MFMA solve phase (DD2_APPLY, DD2_KUP or DD2_BACK) over a unit list, all slice columns.
// single: one state in natural layout (Npad = 1). split = 0: each unit is a
// whole block row (nmb = W/16 <= 32), one workgroup of `waves` waves
// (kDD2WholeRowTiles row tiles each); 1: four units of <= 4 row tiles per workgroup; 4, 8 or 16: one
// unit per workgroup with its k-blocks split over that many waves (launches with
// few units; 16 is taken as 8 for more than two column tiles).
hipError_t launch_dd2_solve(int mode, const DD2Unit* units, int n_units, const double* pool,
                            double* Z, double* Y, int nx, int Npad, bool single, int split,
                            int waves, hipStream_t s);
hipError_t launch_dd2_kup0(const DD2Row* rows, int n_rows, const double* bc, double* Z,
                           const double* Y, int nx, int Npad, hipStream_t s);
// Level-0 eliminated rows, Thomas solves along x for every slice column:
// back = false: Y[r] = D_r^-1 Z[r]; back = true: Z[r] = Y[r] - D_r^-1 (b_r Z[r-1] + c_r Z[r+1]).
// wmax: widest row of the list. per_line: one wave per (row, column) line with
// the row spread over the lanes (affine scans); otherwise one lane per line.
hipError_t launch_dd2_tri0(bool back, const DD2Row* rows, int n_rows, int wmax, bool per_line,
                           const double* tri, const double* bc, double* Z, double* Y, int nx,
                           int Npad, hipStream_t s);
// Natural [N][npts] <-> slice-minor [npts][Npad] (padding columns written as 0).
hipError_t launch_dd2_to_sm(const double* U, double* Zs, long npts, int N, int Npad,
                            hipStream_t s);
hipError_t launch_dd2_from_sm(const double* Zs, double* U, long npts, int N, int Npad,
                              hipStream_t s);
// Douglas-Rachford term S = tau A_k U of colour k (g.rho = colour k's weights,
// g.tx / g.ty / g.tc at the step tau) over the whole grid, slice-minor [node][Npad].
hipError_t launch_dd2_stencil(const DD2Geo& g, const double* U, double* S, int Npad,
                              hipStream_t s);
// Z += a S over n entries.
hipError_t launch_dd2_axpy(double* Z, const double* S, double a, long n, hipStream_t s);
// Zs[p][b] += sum_m gtab[m * gstride + b * steps + t] S_m[p] for b < N.
hipError_t launch_dd2_force_sm(const double* fS, const double* gtab, long gstride, int steps,
                               int t, double* Zs, long npts, int N, int Npad, hipStream_t s);

// ---- adjoint (pr_kernels_adj.hip) ----
hipError_t launch_face_grad_x(const double* nu, const double* W, int nx, int ny, double coef,
                              double* gax, hipStream_t s);
hipError_t launch_face_grad_y(const double* mu, const double* V, int nx, int ny, double coef,
                              double* gay, hipStream_t s);
hipError_t launch_theta_chain(const double* theta, const double* gax, const double* gay, int nx,
                              int ny, double* gth, hipStream_t s);
// Batched face gradients of the parallel-in-time adjoint: g[face] += -coef *
// sum over slices (a_q - a_p)(w_q - w_p), a and w the true values (pending
// chunk correction of a sweep of direction dir applied) of the workspaces
// described by A and Bst (device descriptors; h is A's host copy).
hipError_t launch_grad_faces(int dir, const DimInst* A, const DimInst* Bst, const DimInst& h,
                             double coef, double* g, hipStream_t s);
// Batched 2D transposes of count states: out[s][i][j] = in[s][j][i].
hipError_t launch_transpose_states(const double* in, double* out, int nx, int ny, int count,
                                   hipStream_t s);
// One slice of an interleaved workspace after an x sweep, corrected, natural layout.
hipError_t launch_slice_xcorr(const DimInst* A, const DimInst& h, int slice, double* out,
                              hipStream_t s);

// ---- launchers (pr_kernels_dim.hip) ----
hipError_t launch_faces_from_theta_2d(const double* theta, int nx, int ny, double* ax, double* ay,
                                      hipStream_t s);
hipError_t launch_faces_from_theta_1d(const double* theta, int nx, double* ax, hipStream_t s);
hipError_t launch_factorize(const FactorJob& job, hipStream_t s);
// positions per lane K of a line of n points (smallest power of two with
// 64 K >= n, at most kLineSeg / 64)
int positions_per_lane(int n);
// Segments of a line of n positions for the one-wave-per-line solvers.
int line_segments(int n);
// lane-blocked copy [line][s][c][lane] of line-major factors [line][pos]
hipError_t launch_block_factors(const double* src, int n_lines, int n_pos, double* dst,
                                hipStream_t s);
// Fine factors of one direction with the lines twisted at position mid (mid >=
// n_pos: the plain LU), and the chunk products phi of that factorisation: top
// chunks from the position to the chunk end, bottom chunks from the chunk start
// to the position (phiS: the product over the whole chunk).
hipError_t launch_factorize_twisted(const FactorJob& job, int mid, hipStream_t s);
// out[2 p] = a[p], out[2 p + 1] = b[p] for p < n.
hipError_t launch_interleave_pairs(const double* a, const double* b, long n, double* out,
                                   hipStream_t s);
hipError_t launch_chunk_phi_twisted(const double* G, int n_lines, int n_pos, int M, int kmid,
                                    double* phiC, double* phiS, hipStream_t s);
hipError_t launch_chunk_phi(const double* G, int n_lines, int n_pos, int M, double* phiC,
                            double* phiS, hipStream_t s);
// part: the partitioned sweeps' slice blocks (Lp, Bp, slabp) instead of (L, B, slab).
hipError_t launch_to_interleaved(const DimInst* d_inst, const DimInst& h, const double* U_in,
                                 hipStream_t s, bool part = false);
// with_corr = false: plain transpose (no pending chunk correction).
hipError_t launch_from_interleaved(const DimInst* d_inst, const DimInst& h, double* F_out,
                                   bool with_corr, hipStream_t s, bool part = false);
// sgn = +1 / -1: add / subtract the instance's DR array on load (0: FIE);
// forced: the x sweep adds the step's source term (dir 0 only).
// twisted: two-wave workgroups, the bottom chunks [twx / twy, P) of every line
// eliminated from the line end with the UL factors (see k_fine_sweep).
// grouped (twisted, L = 64, FIE only): workgroups of grouped_lines() lines whose
// work items count line groups of that many lines (k_fine_sweep_g); long_lines:
// some instance of the launch has lines of more than lds_chunk_lines(M) chunks
// (the grouped form then keeps every chunk outer value in the carry slots).
hipError_t launch_fine_sweep(const DimInst* d_insts, const WorkItem* d_work, int n_work, int L,
                             int M, int dir, int has_prev, int step, hipStream_t s, int sgn = 0,
                             bool forced = false, bool twisted = false, bool grouped = false,
                             bool long_lines = false);
int grouped_lines();
// Chunks of M positions whose outer values the fine sweeps keep in LDS.
int lds_chunk_lines(int M);
// Partitioned fine sweeps (k_part_sweep): one workgroup of at most kPartWaves
// waves per (instance, slice block, line) holds the whole line, cut into parts
// of at most kPartMaxPL positions per lane, and writes exact values (no pending
// correction: the next sweep and the final transpose read them as they are).
// Workgroups of 8 waves within 128 registers let two share a compute unit.
constexpr int kPartWaves = 8;
constexpr int kPartMaxPL = 24;  // more positions per lane spill registers
// Positions per part for lines of n positions and slice blocks of at most nb
// slices (0: such a line does not fit one workgroup), and the waves it takes.
int part_positions(int n, int nb);
int part_waves(int n, int Pl, int nb);
// By default the partitioned sweeps serve instances of at most kPartMaxSlices
// slices: with more, the chunked sweeps hold enough line recurrences in flight
// and were measured faster (999^2: partitioned 0.53 against 0.41 of 8 TB/s at
// N = 20, 0.49 against 0.51 at N = 32, 0.44 against 0.48 at N = 48; 1023^2,
// N = 64: 0.43 against 0.53).
constexpr int kPartMaxSlices = 24;
// Slice blocks of the partitioned sweeps for an nx x ny grid and N slices: the
// fewest blocks Bp (of Lp = ceil(N / Bp) slices) with which the lines of both
// directions fit one workgroup, and their positions per part; false if none.
bool part_layout(int nx, int ny, int N, int* Lp, int* Bp, int* plx, int* ply);
// One partitioned sweep of direction dir over the work items (inst, b, line):
// workgroups of `waves` waves, register arrays for pl positions per lane (pl at
// least every item's part length); forced: the x sweep adds the step's source.
hipError_t launch_part_sweep(const DimInst* d_insts, const WorkItem* d_work, int n_work, int dir,
                             int step, int waves, int pl, bool forced, hipStream_t s);
// S = dt A_y U on the slice-interleaved workspace (U with the pending y-sweep
// correction when has_prev) of one instance, slice blocks [b_lo, b_hi), before
// fine step `step` (nothing once the instance has finished its steps).
hipError_t launch_dr_stencil(const DimInst* d_inst, const DimInst& h, int has_prev, int step,
                             int b_lo, int b_hi, hipStream_t s);
// Natural-layout DR helpers for one state: S = dt A_y U and out = U + S (mode 0);
// out = out - S (mode 1).
hipError_t launch_dr_stencil_nat(const DimInst* d_inst, const DimInst& h, const double* U,
                                 double* out, int mode, hipStream_t s);
// Exact line solves of one state, one wave per line (lines longer than
// kLineSeg in segments of kLineSeg positions).
// fine = false uses the coarse factorisation, fine = true the fine one. With
// gtab != NULL the x solve's right-hand side also receives sum_m
// gtab[m * gstride + gidx] S_m (a source table premultiplied by the step).
hipError_t launch_coarse_x(const DimInst* d_inst, const DimInst& h, const double* src, double* dst,
                           bool fine, hipStream_t s, const double* gtab = nullptr, long gidx = 0,
                           long gstride = 0);
// Positions a wave of the one-wave-per-line solvers holds at once (64 lanes x
// 16): longer lines are solved in segments of this length. The fine sweeps keep
// the chunk outer values of lines up to this length in LDS, of longer lines in
// the carry array.
constexpr int kLineSeg = 1024;
constexpr int kCoarseRowsPerBlock = 4;    // x lines per block of the coarse x kernels
constexpr int kCoarseColsPerBlock = 4;    // y lines per block of the coarse y kernels
// Batched coarse sweep: one launch covers every instance's slice n (items of
// instances with n < N and still active). step c of the instance's coarse
// propagation: c == 0 reads U[n] from U_base, later steps the instance's tmp;
// the last step (c == cs-1) applies mode (1: correction + increment, 2:
// initial guess) to U[n+1] / G_old[n] / F[n], the others write tmp.
// The mode-1 increment of each instance goes to its partial maxima (incp,
// zeroed by the caller before the sweep); launch_inc_reduce folds them into
// inc_bits[instance] after the sweep's last launch. seg: some instance of the
// launch has lines of more than one segment (the segmented solve, which holds
// more registers, is then used for the whole launch).
hipError_t launch_coarse_xb(const DimInst* d_insts, const LineItem* items, int n_items, int n,
                            int c, const double* U_base, hipStream_t s, bool seg);
hipError_t launch_coarse_yb(const DimInst* d_insts, const LineItem* items, int n_items, int n,
                            int c, int mode, const double* F_base, double* G_base, double* U_base,
                            hipStream_t s, bool seg);
hipError_t launch_inc_reduce(const DimInst* d_insts, int n_inst, unsigned long long* inc_bits,
                             hipStream_t s);
// Parareal bookkeeping on the device: inc = 0 for active instances (start of
// a correction) and active &= !(inc < tol) (end of a correction).
hipError_t launch_mask_update(const double* inc, int* active, int n, double tol, hipStream_t s);
hipError_t launch_coarse_y(const DimInst* d_inst, const DimInst& h, const double* src, double* dst,
                           bool fine, hipStream_t s);
hipError_t launch_fill_zero(double* p, size_t n, hipStream_t s);
// Source of the DD substeps (every node, since the first stage of a step
// touches all of them): interleaved Z[b][node][l] += sum_m gtab[m][slice*steps
// + step] S_m[node] (forced_z), or one state u += sum_m gtab[m*gstride + gidx] S_m.
hipError_t launch_force_interleaved(const DimInst* d_inst, const DimInst& h, int step,
                                    hipStream_t s);
hipError_t launch_force_state(const DimInst* d_inst, const DimInst& h, double* u,
                              const double* gtab, long gidx, long gstride, hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, size_t n, hipStream_t s);

}  // namespace prk
