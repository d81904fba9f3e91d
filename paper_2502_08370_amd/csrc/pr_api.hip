// Host runtime of the parareal-with-splitting library: validation, workspace,
// factorisation set-up and the launch sequences behind the C ABI of pr.h.
// Method: arXiv 2502.08370 (section 2: splitting and FIE; section 3: parareal).
#include "pr.h"
#include "pr_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

using namespace prk;

namespace {

// Message of the last failure on this thread: a fixed buffer, so that
// recording an error can never throw.
thread_local char g_err[512];

pr_status fail(pr_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

// Every entry point of the C ABI runs its body through guarded(): a C++
// exception (a host allocation inside std::vector, say) becomes a status and
// never unwinds into the caller.
template <class Fn>
pr_status guarded(Fn&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail(PR_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(PR_EDEVICE, "internal error: %s", e.what());
  } catch (...) {
    return fail(PR_EDEVICE, "internal error: unknown C++ exception");
  }
}

#define HIPOK(expr)                                                                  \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(PR_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

int pow2_at_least(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Device buffer owned by the library.
struct DBuf {
  double* p = nullptr;
  size_t n = 0;
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t count) {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = count;
    if (count == 0) return hipSuccess;
    return hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(double));
  }
};

// Device array of a trivially copyable type, owned by the library.
template <class T>
struct DArr {
  T* p = nullptr;
  size_t n = 0;
  ~DArr() {
    if (p) (void)hipFree(p);
  }
  hipError_t upload(const std::vector<T>& v) {
    if (p) {
      (void)hipFree(p);
      p = nullptr;
    }
    n = v.size();
    if (n == 0) return hipSuccess;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), n * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(p, v.data(), n * sizeof(T), hipMemcpyHostToDevice);
  }
};

// Factors of the domain-decomposition substeps at one tau.
struct DDFactorSet {
  DBuf R, G, CHI, PHI, PSIE, CHIA, PHIA;
  DBuf PC0, PP0, PC1, PP1, FC, FP;  // deferred corrections (fine set only)
  DBuf SA, SC, SD;                  // per segment, from its run's factors
  DDFactors view() const {
    return DDFactors{R.p, G.p, CHI.p, PHI.p, PSIE.p, CHIA.p, PHIA.p,
                     PC0.p, PP0.p, PC1.p, PP1.p, FC.p, FP.p, SA.p, SC.p, SD.p};
  }
};

struct Instance {
  pr_problem_desc d;  // copy (pointer members are not retained)
  int npts = 0;
  double dt = 0, tauG = 0;
  size_t off_u0 = 0, off_slices = 0, off_states = 0;
  bool dd = false;
  int Ldef = 0;  // default lane width (sizes the interleaved workspace)
  // dimensional splitting (and, for DD, the transpose fields nx, ny, N, L, B, slab, Z)
  DimInst h{};       // host mirror of the device descriptor
  DBuf ax, ay, theta;
  DBuf fxR, fxG, fyR, fyG, fxPhiC, fyPhiC, fxPhiS, fyPhiS;
  DBuf fxRG, fyRG;  // (r, g) pairs of the fine factors (grouped sweeps)
  DBuf pxRG, pyRG;  // (r, g) pairs of the plain fine LU (partitioned sweeps)
  bool part = false;  // its fine sweeps are partitioned (their output carries no correction)
  int plx0 = 0, ply0 = 0;  // positions per part when they can be (0: the lines do not fit)
  DBuf cxR, cxG, cyR, cyG;
  DBuf cxRb, cxGb, cyRb, cyGb, fxRb, fxGb, fyRb, fyGb;  // lane-blocked copies
  DBuf Z, sigX, sigY, tmp;
  DBuf drS;  // Douglas-Rachford stencil values, shaped like Z
  DBuf fS, fgf, fgc;  // source: spatial factors, step-premultiplied time tables
  // domain decomposition (1D)
  int n_colors = 0;
  std::vector<int> seg_off;   // colour k's segments: [seg_off[k], seg_off[k+1])
  std::vector<int> comp_off;  // colour k's components: [comp_off[k], comp_off[k+1])
  std::vector<int> run_off;   // colour k's carry runs: [run_off[k], run_off[k+1])
  DArr<DDRun> runs;
  DArr<int> comp_run_first, comp_run_count;
  DArr<int> seg_src0, seg_src1, fin_seg;  // pending-correction sources (deferred substeps)
  DArr<int> seg_run;                      // the run of each segment
  DArr<DDRunRec> run_recs;
  DBuf RP, RQ, RU, RV, RW, RY, RX;        // fine (interleaved) run maps and carries
  DBuf RP1, RQ1, RU1, RV1, RW1, RY1, RX1;  // single-state run maps and carries
  DBuf rho, W;
  DArr<DDSeg> segs;
  DArr<int> seg_colour, comp_lo, comp_hi, comp_colour, comp_first, comp_count;
  DDFactorSet ffine, fcoarse;
  DBuf Yp, Xp, Yin, Xin;      // fine (interleaved): slice parts of the carries, final carries
  DBuf Yp1, Xp1;              // single state: slice parts of the carries
  DDInst hdd{}, hdd1{};       // interleaved fine workspace / single state (tmp)
  DDInst* d_dd = nullptr;     // device copies [hdd, hdd1]
  // domain decomposition (2D, vertical strips; dd is also set)
  bool dd2 = false;
  struct Strip2 {
    int colour, col0, w, W;
    long bc0;   // first entry of the strip's coupling vectors in the bc arrays
    long tri0;  // first entry of the strip's level-0 LU (3 W per eliminated row) in the tri arrays
    // factor-pool offsets per level l >= 1 and alive row a (-1: not stored)
    std::vector<std::vector<long>> dinv, m2, m3, bm, cm;
  };
  std::vector<Strip2> strips2;
  struct Phase2 {
    int mode;  // DD2_APPLY / DD2_KUP / DD2_BACK (units) or DD2_KUP0 / DD2_TRI_* (level-0 rows)
    int off, cnt;
    int split;   // see launch_dd2_solve (all slices)
    int split1;  // the same for the single state
    int waves;   // split 0: waves per workgroup
    int wmax;   // level-0 row phases: widest row
  };
  std::vector<std::vector<Phase2>> phases2;  // per colour, in launch order
  DArr<DD2Unit> units2;
  DArr<DD2Row> rows2;
  DBuf pool2f, pool2c, bc2f, bc2c, tri2f, tri2c, rho2, Zs, Ys, Y1;
  DBuf drS2, drS1;  // Douglas-Rachford terms tau A_k U_n of colours k >= 1 (batch / single)
  int Npad2 = 16;
  // adjoint workspace (allocated on the first pr_adjoint call)
  DBuf adjWV, adjCkpt, adjLam, adjMu, adjGax, adjGay;
  // parallel-in-time adjoint: forward snapshots of every step of every slice,
  // their chunk carries, the adjoint workspace, the boundary adjoints
  DBuf pSnap, pSigX, pSigY, pInit, pLam, pSigXa, pSigYa, pBnd, pBndT, pLamIn, pCoefT0, pCoefT1;
  DArr<DimInst> pDesc;
  std::vector<DimInst> pDescHost;  // source of pDesc's stream-ordered upload
  ~Instance() {
    if (d_dd) (void)hipFree(d_dd);
  }
};

}  // namespace

// Fewer one-wave-per-line sweep waves than this (two per SIMD of the 256 CUs):
// twisted sweeps by default.
constexpr long kTwistBelowWaves = 2 * 4 * 256;

struct pr_problem_s {
  std::vector<std::unique_ptr<Instance>> inst;
  // phase timers (pr_profile_control / pr_profile_read)
  bool prof = false;
  bool prof_span = false;  // span mode: one event pair around each loop of launches
  int span_depth = 0;      // open spans (their launches record no events of their own)
  struct Rec {
    int phase;
    hipEvent_t a, b;
    int n;  // launches the interval covers
  };
  std::vector<hipEvent_t> ev_free;
  std::vector<Rec> recs;
  pr_profile acc{};
  size_t tot_u0 = 0, tot_slices = 0, tot_states = 0;
  int M = 20;  // fine-sweep chunk length (PR_OPT_FINE_CHUNK)
  bool twisted = true;  // two-wave twisted fine sweeps (PR_OPT_TWISTED)
  bool grouped = true;  // several lines per workgroup sharing their carry loads (PR_OPT_GROUPED)
  int part_sweeps = 1;  // partitioned sweeps: 0 never, 1 few slices, 2 wherever lines fit (PR_OPT_PARTITIONED)
  DimInst* d_inst = nullptr;  // device descriptors, one per instance
  // grouped work lists per lane width L (index log2 L) and direction
  struct Group {
    int L = 0;
    int dr = 0;                // Douglas-Rachford instances (the sweeps add / subtract S)
    int ft = 0;                // instances with a source term (the x sweep adds it)
    int M = 32;                // chunk length of the group's sweeps
    bool grouped = false;      // workgroups of grouped_lines() lines sharing the carry loads
    bool long_lines = false;   // a member has lines of more than lds_chunk_lines(M) chunks
    std::vector<int> members;  // instances of the group
    WorkItem* d_work[2] = {nullptr, nullptr};
    int n_work[2] = {0, 0};
    std::vector<int> pass_off[2];  // items of pass q: [pass_off[q], pass_off[q+1])
    // partitioned sweeps (every member's lines fit a workgroup): items (inst,
    // b, line), waves per workgroup and register positions per lane
    bool part = false;
    WorkItem* d_pwork[2] = {nullptr, nullptr};
    int n_pwork[2] = {0, 0};
    int pwaves[2] = {0, 0}, ppl[2] = {0, 0};
  };
  int blocks_per_pass = 0;  // 0: every slice block in every launch
  int n_passes = 1;
  int pass_blocks = 1 << 30;  // slice blocks per pass in effect
  std::vector<Group> groups;
  // parareal workspace
  DBuf F, Gold;
  unsigned long long* d_inc = nullptr;
  unsigned long long* d_incp = nullptr;  // per-column-block increment maxima, all instances
  size_t n_incp = 0;
  double* h_inc = nullptr;  // pinned
  int* d_active = nullptr;  // per-instance flags read by every kernel
  // batched coarse sweeps: items of slice index n are [xoff[n], xoff[n+1])
  DArr<LineItem> xitems, yitems;
  std::vector<int> xoff, yoff;
  int Nmax = 0, csmax = 0, max_nx = 1, max_ny = 1;
  bool any_dd = false;
  // captured parareal correction
  bool use_graph = true;
  hipStream_t gstream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double graph_tol = -1.0;
  const double* graph_U = nullptr;
  std::vector<char> graph_active;  // host mask of the domain-decomposition instances baked into the graph
  int lanes_cap = 0;  // 0: each instance uses its default lane width
  pr_problem_s* adjT = nullptr;  // transposed problem of the parallel adjoint
  hipStream_t astream = nullptr;  // its stream (runs beside the forward checkpoints)
  hipEvent_t aev[2] = {nullptr, nullptr};
  ~pr_problem_s() {
    delete adjT;
    for (auto e : aev)
      if (e) (void)hipEventDestroy(e);
    if (astream) (void)hipStreamDestroy(astream);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (gstream) (void)hipStreamDestroy(gstream);
    if (d_active) (void)hipFree(d_active);
    if (d_inst) (void)hipFree(d_inst);
    for (auto& g : groups) {
      for (auto* w : g.d_work)
        if (w) (void)hipFree(w);
      for (auto* w : g.d_pwork)
        if (w) (void)hipFree(w);
    }
    if (d_inc) (void)hipFree(d_inc);
    if (d_incp) (void)hipFree(d_incp);
    if (h_inc) (void)hipHostFree(h_inc);
    for (auto& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : ev_free) (void)hipEventDestroy(e);
  }
};

namespace {

pr_status validate(const pr_problem_desc& d, int idx) {
  if (d.dim != 1 && d.dim != 2) return fail(PR_EINVAL, "instance %d: dim must be 1 or 2", idx);
  if (d.nx < 1 || d.ny < 1) return fail(PR_EINVAL, "instance %d: nx, ny must be >= 1", idx);
  if (d.dim == 1 && d.ny != 1) return fail(PR_EINVAL, "instance %d: ny must be 1 in 1D", idx);
  if ((long)d.nx * d.ny > (1L << 31) / 8) return fail(PR_EINVAL, "instance %d: grid too large", idx);
  if (!(d.T > 0) || !std::isfinite(d.T)) return fail(PR_EINVAL, "instance %d: T must be > 0", idx);
  if (d.n_slices < 1 || d.fine_steps < 1 || d.coarse_steps < 1)
    return fail(PR_EINVAL, "instance %d: n_slices, fine_steps, coarse_steps must be >= 1", idx);
  if (d.fine != PR_FIE && d.fine != PR_DR) return fail(PR_EINVAL, "instance %d: bad fine", idx);
  if (d.fine == PR_DR && d.split == PR_SPLIT_DD && d.dim == 1)
    return fail(PR_EUNSUPPORTED,
                "instance %d: the Douglas-Rachford fine propagator needs a 2D split", idx);
  if (d.split != PR_SPLIT_DIM && d.split != PR_SPLIT_DD)
    return fail(PR_EINVAL, "instance %d: bad split", idx);
  if (d.n_forcing < 0 || d.n_forcing > PR_MAX_FORCING)
    return fail(PR_EINVAL, "instance %d: n_forcing must be in 0..%d", idx, PR_MAX_FORCING);
  if (d.n_forcing > 0 && (!d.forcing_space || !d.forcing_time_fine || !d.forcing_time_coarse))
    return fail(PR_EINVAL, "instance %d: source term arrays are NULL", idx);
  if (d.coef_mode != PR_COEF_FACES && d.coef_mode != PR_COEF_NODAL_LOG)
    return fail(PR_EINVAL, "instance %d: bad coef_mode", idx);
  if (!d.coef_x) return fail(PR_EINVAL, "instance %d: coef_x is NULL", idx);
  if (d.dim == 2 && d.coef_mode == PR_COEF_FACES && !d.coef_y)
    return fail(PR_EINVAL, "instance %d: coef_y is NULL", idx);
  if (!(d.c >= 0) || !std::isfinite(d.c)) return fail(PR_EINVAL, "instance %d: c must be >= 0", idx);
  if (d.split == PR_SPLIT_DIM && d.dim == 1)
    return fail(PR_EUNSUPPORTED, "instance %d: 1D problems use the DD split (one colour, rho = 1)",
                idx);
  if (d.split == PR_SPLIT_DD) {
    if (d.dim == 1 && d.c != 0.0)
      return fail(PR_EUNSUPPORTED, "instance %d: 1D DD splitting needs c = 0", idx);
    if (d.n_colors < 1 || d.n_colors > 64)
      return fail(PR_EINVAL, "instance %d: n_colors must be in 1..64", idx);
    if (!d.rho) return fail(PR_EINVAL, "instance %d: rho is NULL", idx);
    // 1D: one weight per face; 2D: samples on the half grid of x
    const int nr = d.dim == 1 ? d.nx + 1 : 2 * d.nx + 1;
    for (int f = 0; f < nr; f++) {
      double sum = 0.0;
      for (int k = 0; k < d.n_colors; k++) {
        double r = d.rho[(size_t)k * nr + f];
        if (!(r >= 0.0 && r <= 1.0))
          return fail(PR_EINVAL, "instance %d: rho[%d][%d] = %g outside [0, 1]", idx, k, f, r);
        sum += r;
      }
      if (std::fabs(sum - 1.0) > 1e-14)
        return fail(PR_EINVAL, "instance %d: partition of unity sums to %.17g at sample %d", idx,
                    sum, f);
    }
  }
  return PR_OK;
}

// Source term tables of eq. FIE_method / eq. DR_method: S_m copied, unused
// terms zero; g_m premultiplied by the step (dt fine, DT / coarse_steps coarse).
pr_status setup_forcing(Instance& I, const pr_problem_desc& d, hipStream_t s) {
  DimInst& h = I.h;
  h.nforce = d.n_forcing;
  h.fS = h.fgf = h.fgc = nullptr;
  if (d.n_forcing == 0) return PR_OK;
  const size_t npts = (size_t)d.nx * d.ny;
  const size_t nf = (size_t)d.n_slices * d.fine_steps, nc = (size_t)d.n_slices * d.coarse_steps;
  HIPOK(I.fS.alloc(kMaxForcing * npts));
  HIPOK(launch_fill_zero(I.fS.p, I.fS.n, s));
  HIPOK(hipMemcpyAsync(I.fS.p, d.forcing_space, d.n_forcing * npts * sizeof(double),
                       hipMemcpyDeviceToDevice, s));
  std::vector<double> tf(kMaxForcing * nf, 0.0), tc(kMaxForcing * nc, 0.0);
  for (int m = 0; m < d.n_forcing; m++) {
    for (size_t i = 0; i < nf; i++) tf[m * nf + i] = I.dt * d.forcing_time_fine[m * nf + i];
    for (size_t i = 0; i < nc; i++) tc[m * nc + i] = I.tauG * d.forcing_time_coarse[m * nc + i];
  }
  HIPOK(I.fgf.alloc(tf.size()));
  HIPOK(I.fgc.alloc(tc.size()));
  HIPOK(hipMemcpyAsync(I.fgf.p, tf.data(), tf.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPOK(hipMemcpyAsync(I.fgc.p, tc.data(), tc.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPOK(hipStreamSynchronize(s));  // the host tables are released on return
  h.fS = I.fS.p;
  h.fgf = I.fgf.p;
  h.fgc = I.fgc.p;
  return PR_OK;
}

// Split chunk of the twisted fine sweeps: the bottom part of a line starts at
// chunk (P + 1) / 2 (lines of one chunk are not twisted).
void set_twist(DimInst& h, bool twisted) {
  h.twx = (twisted && h.Px >= 2) ? (h.Px + 1) / 2 : h.Px;
  h.twy = (twisted && h.Py >= 2) ? (h.Py + 1) / 2 : h.Py;
}

// Factorisation job of the fine line systems of one direction (tau = dt).
FactorJob fine_job(Instance& I, int dir) {
  const pr_problem_desc& d = I.d;
  const int nx = d.nx, ny = d.ny;
  const double h = dir == 0 ? 1.0 / (nx + 1) : 1.0 / (ny + 1);
  FactorJob j{};
  j.face = dir == 0 ? I.ax.p : I.ay.p;
  j.n_lines = dir == 0 ? ny : nx;
  j.n_pos = dir == 0 ? nx : ny;
  j.face_line_stride = dir == 0 ? nx + 1 : 1;
  j.face_pos_stride = dir == 0 ? 1 : nx;
  j.tau_over_h2 = I.dt / (h * h);
  j.react = I.dt * (d.c / d.dim);
  j.E = nullptr;
  j.R = dir == 0 ? I.fxR.p : I.fyR.p;
  j.G = dir == 0 ? I.fxG.p : I.fyG.p;
  j.pos_major = 0;
  return j;
}

// Fine factors of the sweeps (twisted at chunk twx / twy, plain LU when the
// split chunk is the line's last) and their chunk products phi.
pr_status fine_factors(Instance& I, hipStream_t s) {
  const DimInst& h = I.h;
  const long npts = (long)I.d.nx * I.d.ny;
  HIPOK(launch_factorize_twisted(fine_job(I, 0), h.twx * h.M, s));
  HIPOK(launch_chunk_phi_twisted(I.fxG.p, I.d.ny, I.d.nx, h.M, h.twx, I.fxPhiC.p, I.fxPhiS.p, s));
  HIPOK(launch_interleave_pairs(I.fxR.p, I.fxG.p, npts, I.fxRG.p, s));
  if (I.d.dim == 2) {
    HIPOK(launch_factorize_twisted(fine_job(I, 1), h.twy * h.M, s));
    HIPOK(launch_chunk_phi_twisted(I.fyG.p, I.d.nx, I.d.ny, h.M, h.twy, I.fyPhiC.p, I.fyPhiS.p,
                                   s));
    HIPOK(launch_interleave_pairs(I.fyR.p, I.fyG.p, npts, I.fyRG.p, s));
  }
  return PR_OK;
}

pr_status setup_dim_instance(pr_problem_s* P, Instance& I, hipStream_t s) {
  const pr_problem_desc& d = I.d;
  const int nx = d.nx, ny = d.ny, N = d.n_slices;
  const int M = 16;  // chunk-sized arrays are allocated for the shortest chunk
  const size_t npts = (size_t)nx * ny;
  I.npts = (int)npts;
  I.dt = d.T / d.n_slices / d.fine_steps;
  I.tauG = d.T / d.n_slices / d.coarse_steps;
  // face coefficients
  HIPOK(I.ax.alloc((size_t)ny * (nx + 1)));
  if (d.dim == 2) HIPOK(I.ay.alloc((size_t)(ny + 1) * nx));
  pr_status st = PR_OK;
  (void)st;
  const int Px = (nx + M - 1) / M, Py = (ny + M - 1) / M;
  HIPOK(I.fxR.alloc(npts)); HIPOK(I.fxG.alloc(npts)); HIPOK(I.fxRG.alloc(2 * npts));
  HIPOK(I.pxRG.alloc(2 * npts));
  HIPOK(I.cxR.alloc(npts)); HIPOK(I.cxG.alloc(npts));
  HIPOK(I.fxPhiC.alloc(npts)); HIPOK(I.fxPhiS.alloc((size_t)ny * Px));
  const int Kx = positions_per_lane(nx), Ky = positions_per_lane(ny);
  const int Sx = line_segments(nx), Sy = line_segments(ny);
  const size_t nbx = (size_t)ny * 64 * Kx * Sx, nby = (size_t)nx * 64 * Ky * Sy;
  HIPOK(I.cxRb.alloc(nbx)); HIPOK(I.cxGb.alloc(nbx));
  HIPOK(I.fxRb.alloc(nbx)); HIPOK(I.fxGb.alloc(nbx));
  if (d.dim == 2) {
    HIPOK(I.fyR.alloc(npts)); HIPOK(I.fyG.alloc(npts)); HIPOK(I.fyRG.alloc(2 * npts));
    HIPOK(I.pyRG.alloc(2 * npts));
    HIPOK(I.cyR.alloc(npts)); HIPOK(I.cyG.alloc(npts));
    HIPOK(I.fyPhiC.alloc(npts)); HIPOK(I.fyPhiS.alloc((size_t)nx * Py));
    HIPOK(I.cyRb.alloc(nby)); HIPOK(I.cyGb.alloc(nby));
    HIPOK(I.fyRb.alloc(nby)); HIPOK(I.fyGb.alloc(nby));
  }
  // lanes per slice block: a power of two in [8, 64] (fewer slices are padded)
  const int L = std::min(64, std::max(8, pow2_at_least(N)));
  const int B = (N + L - 1) / L;
  I.Ldef = L;
  DimInst& h = I.h;
  // Douglas-Rachford sweeps hold three arrays per chunk (values, S, carries):
  // they use the short chunk
  const int Mc = d.fine == PR_DR ? kDRChunk : P->M;
  h.nx = nx; h.ny = ny; h.N = N; h.L = L; h.B = B; h.M = Mc;
  h.Px = (nx + Mc - 1) / Mc; h.Py = (ny + Mc - 1) / Mc;
  set_twist(h, P->twisted);
  h.steps = d.fine_steps;
  h.slab = (long)npts * L;
  // slice blocks of the partitioned sweeps (2D FIE only; the workspace holds
  // either layout)
  h.Lp = h.Bp = 0;
  h.slabp = 0;
  if (d.dim == 2 && d.fine == PR_FIE &&
      part_layout(nx, ny, N, &h.Lp, &h.Bp, &I.plx0, &I.ply0))
    h.slabp = (long)npts * h.Lp;
  HIPOK(I.Z.alloc((size_t)std::max(B * L, h.Bp * h.Lp) * npts));
  HIPOK(I.sigX.alloc((size_t)B * ny * Px * L));
  if (d.dim == 2) HIPOK(I.sigY.alloc((size_t)B * nx * Py * L));
  HIPOK(I.tmp.alloc(npts));
  h.Z = I.Z.p; h.sigX = I.sigX.p; h.sigY = I.sigY.p;
  h.dr = d.fine == PR_DR;
  h.drS = nullptr;
  h.ay = I.ay.p;
  if (h.dr) {
    // S = dt A_y U with A_y = D_y a D_y - c/2 (the reaction shared by the two terms)
    HIPOK(I.drS.alloc((size_t)B * npts * L));
    h.drS = I.drS.p;
    const double hy = 1.0 / (ny + 1);
    h.dr_coef = I.dt / (hy * hy);
    h.dr_react = I.dt * (d.c / 2.0);
  }
  h.fxR = I.fxR.p; h.fxG = I.fxG.p;
  h.fyR = I.fyR.p; h.fyG = I.fyG.p;
  h.fxRG = I.fxRG.p; h.fyRG = I.fyRG.p;
  h.pxRG = I.pxRG.p; h.pyRG = I.pyRG.p;
  h.plx = h.ply = 0;
  h.fxPhiC = I.fxPhiC.p; h.fyPhiC = I.fyPhiC.p; h.fxPhiS = I.fxPhiS.p; h.fyPhiS = I.fyPhiS.p;
  h.Kx = Kx; h.Ky = Ky; h.Sx = Sx; h.Sy = Sy;
  h.cxRb = I.cxRb.p; h.cxGb = I.cxGb.p; h.cyRb = I.cyRb.p; h.cyGb = I.cyGb.p;
  h.fxRb = I.fxRb.p; h.fxGb = I.fxGb.p; h.fyRb = I.fyRb.p; h.fyGb = I.fyGb.p;
  h.tmp = I.tmp.p;
  return setup_forcing(I, d, s);
}

// Factorisations of I - tau A_x, I - tau A_y at tau = dt (fine, line-major, with
// chunk phi) and tau = DT / coarse_steps (coarse, position-major).
pr_status factorize_instance(pr_problem_s* P, Instance& I, const double* coef_x,
                             const double* coef_y, hipStream_t s) {
  const pr_problem_desc& d = I.d;
  const int nx = d.nx, ny = d.ny, M = I.h.M;
  if (d.coef_mode == PR_COEF_NODAL_LOG) {
    const size_t nth = (size_t)(nx + 2) * (ny + 2);
    if (I.theta.n != nth) HIPOK(I.theta.alloc(nth));
    HIPOK(hipMemcpyAsync(I.theta.p, coef_x, nth * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (d.dim == 2)
      HIPOK(launch_faces_from_theta_2d(coef_x, nx, ny, I.ax.p, I.ay.p, s));
    else
      HIPOK(launch_faces_from_theta_1d(coef_x, nx, I.ax.p, s));
  } else {
    HIPOK(hipMemcpyAsync(I.ax.p, coef_x, I.ax.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (d.dim == 2)
      HIPOK(hipMemcpyAsync(I.ay.p, coef_y, I.ay.n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  const double hx = 1.0 / (nx + 1), hy = 1.0 / (ny + 1);
  const double react = d.c / d.dim;
  for (int coarse = 0; coarse < 2; coarse++) {
    const double tau = coarse ? I.tauG : I.dt;
    FactorJob jx{};
    jx.face = I.ax.p; jx.n_lines = ny; jx.n_pos = nx;
    jx.face_line_stride = nx + 1; jx.face_pos_stride = 1;
    jx.tau_over_h2 = tau / (hx * hx); jx.react = tau * react;
    jx.E = nullptr; jx.R = coarse ? I.cxR.p : I.fxR.p;
    jx.G = coarse ? I.cxG.p : I.fxG.p; jx.pos_major = 0;
    HIPOK(launch_factorize(jx, s));
    if (!coarse) HIPOK(launch_interleave_pairs(jx.R, jx.G, (long)nx * ny, I.pxRG.p, s));
    HIPOK(launch_block_factors(jx.R, ny, nx, coarse ? I.cxRb.p : I.fxRb.p, s));
    HIPOK(launch_block_factors(jx.G, ny, nx, coarse ? I.cxGb.p : I.fxGb.p, s));
    if (d.dim == 2) {
      FactorJob jy{};
      jy.face = I.ay.p; jy.n_lines = nx; jy.n_pos = ny;
      jy.face_line_stride = 1; jy.face_pos_stride = nx;
      jy.tau_over_h2 = tau / (hy * hy); jy.react = tau * react;
      jy.E = nullptr; jy.R = coarse ? I.cyR.p : I.fyR.p;
      jy.G = coarse ? I.cyG.p : I.fyG.p; jy.pos_major = 0;
      HIPOK(launch_factorize(jy, s));
      if (!coarse) HIPOK(launch_interleave_pairs(jy.R, jy.G, (long)nx * ny, I.pyRG.p, s));
      HIPOK(launch_block_factors(jy.R, nx, ny, coarse ? I.cyRb.p : I.fyRb.p, s));
      HIPOK(launch_block_factors(jy.G, nx, ny, coarse ? I.cyGb.p : I.fyGb.p, s));
    }
  }
  (void)M;
  // the fine sweeps' factors: twisted at the instance's split chunk (the lane-
  // blocked copies above keep the plain LU)
  return fine_factors(I, s);
}

enum { PH_FINE = 0, PH_TRANSPOSE = 1, PH_COARSE_X = 2, PH_COARSE_Y = 3, PH_OTHER = 4,
       PH_COARSE = 5 };

hipEvent_t take_event(pr_problem_s* P) {
  if (!P->ev_free.empty()) {
    hipEvent_t e = P->ev_free.back();
    P->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records a start event on construction and a stop event on destruction when
// profiling is on.
struct PhaseTimer {
  pr_problem_s* P;
  int phase;
  hipStream_t s;
  hipEvent_t a = nullptr;
  PhaseTimer(pr_problem_s* P_, int ph, hipStream_t s_) : P(P_), phase(ph), s(s_) {
    if (!P->prof || P->span_depth > 0) return;
    a = take_event(P);
    if (a && hipEventRecord(a, s) != hipSuccess) a = nullptr;
  }
  ~PhaseTimer() {
    if (!a) return;
    hipEvent_t b = take_event(P);
    if (!b || hipEventRecord(b, s) != hipSuccess) {
      P->ev_free.push_back(a);
      if (b) P->ev_free.push_back(b);
      return;
    }
    P->recs.push_back({phase, a, b, 1});
  }
};

// Span-mode timer: one event pair around a loop of launches, which count
// themselves with add(); the per-launch timers inside it record nothing. The
// interval includes the gaps between the launches, so its mean per launch is an
// upper bound of a launch's duration, at a cost of two events per loop instead
// of two per launch.
struct PhaseSpan {
  pr_problem_s* P;
  int phase;
  hipStream_t s;
  hipEvent_t a = nullptr;
  int n = 0;
  PhaseSpan(pr_problem_s* P_, int ph, hipStream_t s_) : P(P_), phase(ph), s(s_) {
    if (!P->prof || !P->prof_span) return;
    a = take_event(P);
    if (a && hipEventRecord(a, s) != hipSuccess) a = nullptr;
    if (a) P->span_depth++;
  }
  void add(int k = 1) { n += k; }
  ~PhaseSpan() {
    if (!a) return;
    P->span_depth--;
    hipEvent_t b = take_event(P);
    if (!b || hipEventRecord(b, s) != hipSuccess || n == 0) {
      P->ev_free.push_back(a);
      if (b) P->ev_free.push_back(b);
      return;
    }
    P->recs.push_back({phase, a, b, n});
  }
};

pr_status set_all_active(pr_problem_s* P, hipStream_t s);
pr_status build_schedules(pr_problem_s* P);

// Sequential fine solve of one dimensional-splitting instance: U[0] = u0,
// U[n+1] = F^s(U[n]), every fine step an exact x then y line solve.
pr_status seq_fine_dim(pr_problem_s* P, int i, const double* u0, double* U, hipStream_t s);

// Domain-decomposition instance: components are the maximal runs of faces with
// rho_k > 0 (node range [first face - 1, last face] clipped to the grid),
// cut into segments of kDDSeg nodes.
pr_status setup_dd_instance(pr_problem_s* P, Instance& I, const double* rho_host, hipStream_t s) {
  (void)P;
  const pr_problem_desc& d = I.d;
  const int n = d.nx, N = d.n_slices, K = d.n_colors;
  I.dd = true;
  I.n_colors = K;
  I.npts = n;
  I.dt = d.T / d.n_slices / d.fine_steps;
  I.tauG = d.T / d.n_slices / d.coarse_steps;
  std::vector<int> clo, chi, ccol, cfirst, ccount, scol;
  std::vector<DDSeg> segs;
  I.seg_off.assign(1, 0);
  I.comp_off.assign(1, 0);
  // components of every colour
  for (int k = 0; k < K; k++) {
    const double* rk = rho_host + (size_t)k * (n + 1);
    int f = 0;
    while (f <= n) {
      if (!(rk[f] > 0.0)) {
        f++;
        continue;
      }
      const int fa = f;
      while (f <= n && rk[f] > 0.0) f++;
      const int fb = f - 1;
      const int lo = std::max(fa - 1, 0), hi = std::min(fb, n - 1);
      if (lo > hi) continue;
      clo.push_back(lo); chi.push_back(hi); ccol.push_back(k);
    }
    I.comp_off.push_back((int)clo.size());
  }
  // Segments: every component cut at a common set of points (multiples of
  // kDDSeg and every component end of every colour), so that segments of
  // different colours covering a node span the same node range.
  std::vector<int> cuts;
  for (int x = 0; x < n; x += kDDSeg) cuts.push_back(x);
  for (size_t c = 0; c < clo.size(); c++) {
    cuts.push_back(clo[c]);
    cuts.push_back(chi[c] + 1);
  }
  std::sort(cuts.begin(), cuts.end());
  cuts.erase(std::unique(cuts.begin(), cuts.end()), cuts.end());
  std::vector<std::vector<int>> starts(K);  // segment starts per colour (sorted)
  for (int k = 0; k < K; k++) {
    for (int c = I.comp_off[k]; c < I.comp_off[k + 1]; c++) {
      cfirst.push_back((int)segs.size());
      auto it = std::upper_bound(cuts.begin(), cuts.end(), clo[c]);
      int a = clo[c];
      while (a <= chi[c]) {
        const int b = (it != cuts.end() && *it <= chi[c]) ? *it : chi[c] + 1;
        segs.push_back(DDSeg{a, b - a, c, k});
        scol.push_back(k);
        starts[k].push_back(a);
        a = b;
        if (it != cuts.end()) ++it;
      }
      ccount.push_back((int)segs.size() - cfirst.back());
    }
    I.seg_off.push_back((int)segs.size());
  }
  const int n_segs = (int)segs.size();
  // Pending-correction sources of the deferred fine substeps. When colour k
  // loads a node, the node still carries the correction of the last substep
  // that solved it: the largest colour k' < k covering it in the same step
  // ("fresh"), else the largest colour covering it in the previous step
  // ("stale", colour k itself at the latest). Segments are aligned, so the
  // source is one segment per segment. After the last step every node
  // carries the correction of the largest colour covering it.
  auto seg_at = [&](int k, int a) -> int {  // colour k's segment starting at a, or -1
    auto it = std::lower_bound(starts[k].begin(), starts[k].end(), a);
    if (it == starts[k].end() || *it != a) return -1;
    return I.seg_off[k] + (int)(it - starts[k].begin());
  };
  std::vector<int> sfresh(n_segs, -1), sstale(n_segs, -1), fin(n, -1);
  for (int k = 0; k < K; k++)
    for (int si = I.seg_off[k]; si < I.seg_off[k + 1]; si++) {
      for (int k2 = k - 1; k2 >= 0 && sfresh[si] < 0; k2--) sfresh[si] = seg_at(k2, segs[si].lo);
      for (int k2 = K - 1; k2 >= k && sstale[si] < 0; k2--) sstale[si] = seg_at(k2, segs[si].lo);
    }
  for (int k = K - 1; k >= 0; k--)
    for (int si = I.seg_off[k]; si < I.seg_off[k + 1]; si++)
      for (int x = segs[si].lo; x < segs[si].lo + segs[si].len; x++)
        if (fin[x] < 0) fin[x] = si;
  std::vector<int> src1(n_segs);
  for (int si = 0; si < n_segs; si++) src1[si] = sfresh[si] >= 0 ? sfresh[si] : sstale[si];
  HIPOK(I.seg_src0.upload(sfresh));
  HIPOK(I.seg_src1.upload(src1));
  HIPOK(I.fin_seg.upload(fin));
  // carry runs: kDDRun consecutive segments of one component
  std::vector<DDRun> runs;
  std::vector<int> crfirst, crcount;
  I.run_off.assign(1, 0);
  for (int k = 0; k < K; k++) {
    for (int c = I.comp_off[k]; c < I.comp_off[k + 1]; c++) {
      crfirst.push_back((int)runs.size());
      for (int q = 0; q < ccount[c]; q += kDDRun)
        runs.push_back(DDRun{cfirst[c] + q, std::min(kDDRun, ccount[c] - q)});
      crcount.push_back((int)runs.size() - crfirst.back());
    }
    I.run_off.push_back((int)runs.size());
  }
  const int n_runs = (int)runs.size();
  std::vector<int> srun(std::max(n_segs, 1), 0);  // the run of each segment
  for (int r = 0; r < n_runs; r++)
    for (int t = 0; t < runs[r].len; t++) srun[runs[r].seg0 + t] = r;
  HIPOK(I.seg_run.upload(srun));
  std::vector<DDRunRec> recs(std::max(n_runs, 1));
  for (int r = 0; r < n_runs; r++) {
    DDRunRec& q = recs[r];
    q = DDRunRec{};
    q.seg0 = runs[r].seg0;
    q.len = runs[r].len;
    for (int t = 0; t < kDDRun; t++) {
      const int si = q.seg0 + std::min(t, q.len - 1);  // clamped past the run's end
      q.lo[t] = segs[si].lo;
      q.cnt[t] = t < q.len ? segs[si].len : 0;
      q.src[0][t] = sfresh[si];
      q.src[1][t] = src1[si];
      q.srun[0][t] = sfresh[si] >= 0 ? srun[sfresh[si]] : 0;
      q.srun[1][t] = src1[si] >= 0 ? srun[src1[si]] : 0;
    }
  }
  HIPOK(I.run_recs.upload(recs));
  HIPOK(I.runs.upload(runs));
  HIPOK(I.comp_run_first.upload(crfirst));
  HIPOK(I.comp_run_count.upload(crcount));
  HIPOK(I.segs.upload(segs));
  HIPOK(I.seg_colour.upload(scol));
  HIPOK(I.comp_lo.upload(clo)); HIPOK(I.comp_hi.upload(chi)); HIPOK(I.comp_colour.upload(ccol));
  HIPOK(I.comp_first.upload(cfirst)); HIPOK(I.comp_count.upload(ccount));
  HIPOK(I.rho.alloc((size_t)K * (n + 1)));
  HIPOK(hipMemcpyAsync(I.rho.p, rho_host, I.rho.n * sizeof(double), hipMemcpyHostToDevice, s));
  HIPOK(I.ax.alloc((size_t)n + 1));
  HIPOK(I.W.alloc((size_t)K * (n + 1)));
  for (DDFactorSet* fs : {&I.ffine, &I.fcoarse}) {
    for (DBuf* b : {&fs->R, &fs->G, &fs->CHI, &fs->PHI}) {
      HIPOK(b->alloc((size_t)K * n));
      HIPOK(launch_fill_zero(b->p, b->n, s));
    }
    for (DBuf* b : {&fs->PSIE, &fs->CHIA, &fs->PHIA, &fs->SA, &fs->SC, &fs->SD})
      HIPOK(b->alloc(std::max(n_segs, 1)));
  }
  for (DBuf* b : {&I.ffine.PC0, &I.ffine.PP0, &I.ffine.PC1, &I.ffine.PP1}) {
    HIPOK(b->alloc((size_t)K * n));
    HIPOK(launch_fill_zero(b->p, b->n, s));
  }
  for (DBuf* b : {&I.ffine.FC, &I.ffine.FP}) HIPOK(b->alloc((size_t)n));
  const int L = std::min(64, std::max(8, pow2_at_least(N)));
  const int B = (N + L - 1) / L;
  HIPOK(I.Z.alloc((size_t)B * n * L));
  HIPOK(I.tmp.alloc(n));
  for (DBuf* b : {&I.Yp, &I.Xp, &I.Yin, &I.Xin})
    HIPOK(b->alloc((size_t)B * std::max(n_segs, 1) * L));
  for (DBuf* b : {&I.Yp1, &I.Xp1}) HIPOK(b->alloc(std::max(n_segs, 1)));
  for (DBuf* b : {&I.RP, &I.RQ, &I.RU, &I.RV, &I.RW, &I.RY, &I.RX})
    HIPOK(b->alloc((size_t)B * std::max(n_runs, 1) * L));
  for (DBuf* b : {&I.RP1, &I.RQ1, &I.RU1, &I.RV1, &I.RW1, &I.RY1, &I.RX1})
    HIPOK(b->alloc(std::max(n_runs, 1)));
  DDInst& h = I.hdd;
  h.n = n; h.N = N; h.L = L; h.B = B; h.n_colors = K; h.n_segs = n_segs;
  h.slab = (long)n * L; h.Z = I.Z.p; h.segs = I.segs.p;
  h.Yin = I.Yin.p; h.Xin = I.Xin.p;
  h.Yp = I.Yp.p; h.Xp = I.Xp.p;
  h.n_runs = n_runs; h.runs = I.runs.p;
  h.seg_src0 = I.seg_src0.p; h.seg_src1 = I.seg_src1.p; h.fin_seg = I.fin_seg.p;
  h.seg_run = I.seg_run.p; h.run_recs = I.run_recs.p;
  h.RP = I.RP.p; h.RQ = I.RQ.p; h.RU = I.RU.p; h.RV = I.RV.p; h.RW = I.RW.p;
  h.RY = I.RY.p; h.RX = I.RX.p;
  DDInst& h1 = I.hdd1;
  h1 = h;
  h1.N = 1; h1.L = 1; h1.B = 1; h1.slab = n; h1.Z = I.tmp.p;
  h1.Yin = h1.Xin = nullptr;
  h1.Yp = I.Yp1.p; h1.Xp = I.Xp1.p;
  h1.RP = I.RP1.p; h1.RQ = I.RQ1.p; h1.RU = I.RU1.p; h1.RV = I.RV1.p; h1.RW = I.RW1.p;
  h1.RY = I.RY1.p; h1.RX = I.RX1.p;
  HIPOK(hipMalloc(reinterpret_cast<void**>(&I.d_dd), 2 * sizeof(DDInst)));
  DDInst both[2] = {h, h1};
  HIPOK(hipMemcpy(I.d_dd, both, sizeof(both), hipMemcpyHostToDevice));
  // transpose view (natural [slice][node] <-> interleaved [b][node][l])
  DimInst& t = I.h;
  t.nx = n; t.ny = 1; t.N = N; t.L = L; t.B = B; t.M = 1; t.Px = 1; t.Py = 1;
  t.steps = d.fine_steps; t.slab = (long)n * L; t.Z = I.Z.p; t.tmp = I.tmp.p;
  t.npts = n;
  return setup_forcing(I, d, s);
}

pr_status factorize_dd_instance(Instance& I, const double* coef_x, hipStream_t s) {
  const pr_problem_desc& d = I.d;
  const int n = d.nx, K = I.n_colors;
  if (d.coef_mode == PR_COEF_NODAL_LOG)
    HIPOK(launch_faces_from_theta_1d(coef_x, n, I.ax.p, s));
  else
    HIPOK(hipMemcpyAsync(I.ax.p, coef_x, I.ax.n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPOK(launch_dd_faces(I.rho.p, I.ax.p, n, K, I.W.p, s));
  const double h = 1.0 / (n + 1);
  const int n_comps = I.comp_off.back(), n_segs = I.seg_off.back();
  for (int coarse = 0; coarse < 2; coarse++) {
    DDFactorSet& fs = coarse ? I.fcoarse : I.ffine;
    const double tau = coarse ? I.tauG : I.dt;
    HIPOK(launch_dd_factorize(I.W.p, n, I.comp_lo.p, I.comp_hi.p, I.comp_colour.p, n_comps,
                              tau / (h * h), fs.R.p, fs.G.p, s));
    HIPOK(launch_dd_segfactors(I.segs.p, I.seg_colour.p, n_segs, n, fs.R.p, fs.G.p,
                               fs.CHI.p, fs.PHI.p, fs.PSIE.p, fs.CHIA.p, fs.PHIA.p, s));
    HIPOK(launch_dd_runfactors(I.d_dd, I.hdd, fs.view(), fs.SA.p, fs.SC.p, fs.SD.p, s));
  }
  DDFactorSet& ff = I.ffine;
  HIPOK(launch_dd_pending(I.d_dd, I.hdd, ff.view(), ff.PC0.p, ff.PP0.p, ff.PC1.p, ff.PP1.p,
                          ff.FC.p, ff.FP.p, s));
  return PR_OK;
}

// One FIE step (eq. FIE_method) of the DD splitting: colours in order, each
// colour's components solved by segment solves, carry scans and corrections.
// which = 0: interleaved fine workspace, whose corrections are deferred to the
// next load (step = the step's index; the last step's are applied by
// launch_dd_from_interleaved); which = 1: the single state in tmp, corrected
// in place.
pr_status dd_fie_step(pr_problem_s* P, Instance& I, bool coarse, int which, int step,
                      hipStream_t s) {
  const DDInst* dI = I.d_dd + which;
  const DDInst& h = which ? I.hdd1 : I.hdd;
  const DDFactors f = (coarse ? I.fcoarse : I.ffine).view();
  const bool defer = which == 0;
  for (int k = 0; k < I.n_colors; k++) {
    const int sb = I.seg_off[k], sc = I.seg_off[k + 1] - sb;
    const int cb = I.comp_off[k], cc = I.comp_off[k + 1] - cb;
    const int rb = I.run_off[k], rc = I.run_off[k + 1] - rb;
    PhaseTimer pt(P, which ? PH_COARSE_X : PH_FINE, s);
    HIPOK(launch_dd_local(dI, h, f, k, sb, sc, rb, rc, step > 0, s));
    HIPOK(launch_dd_carries(dI, h, f, rb, rc, I.comp_run_first.p + cb, I.comp_run_count.p + cb, cc,
                            s));
    if (!defer) HIPOK(launch_dd_correct(dI, h, f, k, sb, sc, s));
  }
  return PR_OK;
}

// ---------------------------------------------------------------------------
// 2D domain decomposition (vertical strips). Strips of colour k are the maximal
// runs of columns where rho_k is nonzero on the node or on one of its x-faces.

// Factor-pool slots of one strip: every dense matrix the block cyclic
// reduction stores, W x W each (levels >= 1; level 0 keeps the LU of its
// tridiagonal blocks instead). Level l has n_l = ny >> l alive rows
// r = 2^l (a+1) - 1.
long dd2_slots(Instance::Strip2& S, int ny, long next) {
  const long sz = (long)S.W * S.W;
  S.dinv.clear(); S.m2.clear(); S.m3.clear(); S.bm.clear(); S.cm.clear();
  for (int l = 0; (ny >> l) > 0; l++) {
    const int n = ny >> l;
    std::vector<long> di(n, -1), m2(n, -1), m3(n, -1), bm(n, -1), cm(n, -1);
    for (int a = 0; a < n; a++) {
      if (l == 0) continue;
      if (a % 2 == 0) {
        di[a] = next; next += sz;
        if (a >= 1) { m2[a] = next; next += sz; }
        if (a + 1 < n) { m3[a] = next; next += sz; }
      } else {
        bm[a] = next; next += sz;
        if (a + 1 < n) { cm[a] = next; next += sz; }
      }
    }
    S.dinv.push_back(di); S.m2.push_back(m2); S.m3.push_back(m3);
    S.bm.push_back(bm); S.cm.push_back(cm);
  }
  return next;
}

// Launches with fewer units than this split each unit's k-range over the four
// waves of a workgroup, below kDD2Split8Units (all slices) or kDD2Split8Single
// (single state) over eight, and below the Split16 counts over sixteen
// (measured).
constexpr int kDD2SplitUnits = 4096;
// Launches with at least this many four-tile units take one workgroup per block row.
constexpr int kDD2WholeRowUnits = 2048;
constexpr int kDD2Split8Units = 640;
constexpr int kDD2Split8Single = 1280;
constexpr int kDD2Split16Units = 320;
constexpr int kDD2Split16Single = 640;

// Launch schedule of one colour: forward levels (eliminated rows y = D^-1 r,
// then kept rows r -= B y_- + C y_+), then back substitution from the top
// level down. Each output row block is split into units of nmb row tiles;
// launches with few row blocks use smaller units so more waves share them.
void dd2_schedule(Instance& I, int colour, std::vector<DD2Unit>& units,
                  std::vector<DD2Row>& rows) {
  const int ny = I.d.ny;
  std::vector<Instance::Phase2> ph;
  auto add_units = [&](int mode, const std::vector<DD2Unit>& tasks) {
    if (tasks.empty()) return;
    long tiles4 = 0;
    int max_tiles = 0;
    for (auto& t : tasks) {
      tiles4 += (t.W / 16 + 3) / 4;
      max_tiles = std::max(max_tiles, t.W / 16);
    }
    const int off = (int)units.size();
    if (tiles4 >= kDD2WholeRowUnits && max_tiles <= 32) {
      // many units: one workgroup per block row
      for (auto t : tasks) {
        t.mb0 = 0;
        t.nmb = t.W / 16;
        units.push_back(t);
      }
      ph.push_back({mode, off, (int)units.size() - off, 0, 0,
                    (max_tiles + kDD2WholeRowTiles - 1) / kDD2WholeRowTiles, 0});
      return;
    }
    const int nmb = std::min(kDD2SplitTiles, tiles4 >= 512 ? 4 : (tiles4 >= 128 ? 2 : 1));
    for (auto t : tasks)
      for (int mb = 0; mb < t.W / 16; mb += nmb) {
        t.mb0 = mb;
        t.nmb = std::min(nmb, t.W / 16 - mb);
        units.push_back(t);
      }
    const int cnt = (int)units.size() - off;
    const int split = cnt < kDD2SplitUnits ? 4 : 1;
    ph.push_back({mode, off, cnt,
                  cnt < kDD2Split16Units ? 16 : (cnt < kDD2Split8Units ? 8 : split),
                  cnt < kDD2Split16Single ? 16 : (cnt < kDD2Split8Single ? 8 : split), 0, 0});
  };
  int L = 0;
  while ((ny >> L) > 0) L++;
  for (int l = 0; l < L; l++) {
    const int n = ny >> l, st = 1 << l;
    std::vector<DD2Unit> ap, kup;
    std::vector<DD2Row> e0, k0;
    for (auto& S : I.strips2) {
      if (S.colour != colour) continue;
      for (int a = 0; a < n; a++) {
        const int r = st * (a + 1) - 1;
        DD2Unit u{S.col0, S.w, S.W, r, 0, 0, -1, -1, -1, -1, -1, S.bc0 + (long)r * 2 * S.W};
        if (l == 0) {
          // level 0: row r = a, eliminated (even a, Thomas with its LU) or kept
          DD2Row R{S.col0, S.w, S.W, r, r >= 1 ? r - 1 : -1, r + 1 < ny ? r + 1 : -1,
                   S.bc0 + (long)r * 2 * S.W, -1};
          if (a % 2 == 0) {
            R.tri = S.tri0 + (long)(a / 2) * 3 * S.W;
            e0.push_back(R);
          } else {
            k0.push_back(R);
          }
        } else if (a % 2 == 0) {
          u.A0 = S.dinv[l][a];
          ap.push_back(u);
        } else {
          u.rowm = r - st; u.A1 = S.bm[l][a];
          if (a + 1 < n) { u.rowp = r + st; u.A2 = S.cm[l][a]; }
          kup.push_back(u);
        }
      }
    }
    auto add_rows = [&](int mode, const std::vector<DD2Row>& rs) {
      if (rs.empty()) return;
      int wm = 1;
      for (auto& r : rs) wm = std::max(wm, r.w);
      ph.push_back({mode, (int)rows.size(), (int)rs.size(), 0, 0, 0, wm});
      rows.insert(rows.end(), rs.begin(), rs.end());
    };
    add_rows(DD2_TRI_APPLY, e0);
    add_units(DD2_APPLY, ap);
    add_rows(DD2_KUP0, k0);
    add_units(DD2_KUP, kup);
  }
  for (int l = L - 1; l >= 0; l--) {
    const int n = ny >> l, st = 1 << l;
    std::vector<DD2Unit> bk;
    std::vector<DD2Row> b0;
    for (auto& S : I.strips2) {
      if (S.colour != colour) continue;
      for (int a = 0; a < n; a += 2) {
        const int r = st * (a + 1) - 1;
        if (l == 0) {
          b0.push_back(DD2Row{S.col0, S.w, S.W, r, r >= 1 ? r - 1 : -1, r + 1 < ny ? r + 1 : -1,
                              S.bc0 + (long)r * 2 * S.W, S.tri0 + (long)(a / 2) * 3 * S.W});
          continue;
        }
        DD2Unit u{S.col0, S.w, S.W, r, 0, 0, -1, -1, -1, -1, -1, S.bc0 + (long)r * 2 * S.W};
        if (a >= 1) { u.rowm = r - st; u.A1 = S.m2[l][a]; }
        if (a + 1 < n) { u.rowp = r + st; u.A2 = S.m3[l][a]; }
        bk.push_back(u);
      }
    }
    if (l == 0) {
      int wm = 1;
      for (auto& r : b0) wm = std::max(wm, r.w);
      ph.push_back({DD2_TRI_BACK, (int)rows.size(), (int)b0.size(), 0, 0, 0, wm});
      rows.insert(rows.end(), b0.begin(), b0.end());
    } else {
      add_units(DD2_BACK, bk);
    }
  }
  I.phases2[colour] = ph;
}

pr_status setup_dd2_instance(Instance& I, const double* rho_host, hipStream_t s) {
  const pr_problem_desc& d = I.d;
  const int nx = d.nx, ny = d.ny, N = d.n_slices, K = d.n_colors;
  const size_t npts = (size_t)nx * ny;
  I.dd = true;
  I.dd2 = true;
  I.n_colors = K;
  I.npts = (int)npts;
  I.dt = d.T / d.n_slices / d.fine_steps;
  I.tauG = d.T / d.n_slices / d.coarse_steps;
  I.strips2.clear();
  for (int k = 0; k < K; k++) {
    const double* r = rho_host + (size_t)k * (2 * nx + 1);
    auto active = [&](int i) { return r[2 * i] > 0.0 || r[2 * i + 1] > 0.0 || r[2 * i + 2] > 0.0; };
    int i = 0;
    while (i < nx) {
      if (!active(i)) { i++; continue; }
      int j = i;
      while (j < nx && active(j)) j++;
      Instance::Strip2 S;
      S.colour = k; S.col0 = i; S.w = j - i; S.W = (S.w + 15) / 16 * 16; S.bc0 = 0;
      if (S.W > kDD2MaxW)
        return fail(PR_EUNSUPPORTED,
                    "2D DD strip of %d columns (at most %d; use more strips per subdomain)", S.w,
                    kDD2MaxW);
      I.strips2.push_back(S);
      i = j;
    }
  }
  long next = 0, bcn = 0, trin = 0;
  for (auto& S : I.strips2) {
    next = dd2_slots(S, ny, next);
    S.bc0 = bcn;
    bcn += (long)ny * 2 * S.W;
    S.tri0 = trin;
    trin += (long)((ny + 1) / 2) * 3 * S.W;
  }
  std::vector<DD2Unit> units;
  std::vector<DD2Row> rows;
  I.phases2.assign(K, {});
  for (int k = 0; k < K; k++) dd2_schedule(I, k, units, rows);
  HIPOK(I.units2.upload(units));
  HIPOK(I.rows2.upload(rows));
  HIPOK(I.pool2f.alloc((size_t)std::max(1L, next)));
  HIPOK(I.pool2c.alloc((size_t)std::max(1L, next)));
  HIPOK(I.bc2f.alloc((size_t)std::max(1L, bcn)));
  HIPOK(I.bc2c.alloc((size_t)std::max(1L, bcn)));
  HIPOK(I.tri2f.alloc((size_t)std::max(1L, trin)));
  HIPOK(I.tri2c.alloc((size_t)std::max(1L, trin)));
  HIPOK(I.rho2.alloc((size_t)K * (2 * nx + 1)));
  HIPOK(hipMemcpy(I.rho2.p, rho_host, I.rho2.n * sizeof(double), hipMemcpyHostToDevice));
  HIPOK(I.ax.alloc((size_t)ny * (nx + 1)));
  HIPOK(I.ay.alloc((size_t)(ny + 1) * nx));
  I.Npad2 = (N + 15) / 16 * 16;
  HIPOK(I.Zs.alloc(npts * I.Npad2));
  HIPOK(I.Ys.alloc(npts * I.Npad2));
  HIPOK(I.Y1.alloc(npts));
  HIPOK(I.tmp.alloc(npts));
  if (d.fine == PR_DR && K > 1) {
    HIPOK(I.drS2.alloc((size_t)(K - 1) * npts * I.Npad2));
    HIPOK(I.drS1.alloc((size_t)(K - 1) * npts));
  }
  DimInst& h = I.h;
  h.nx = nx; h.ny = ny; h.N = N; h.L = 1; h.B = 1; h.M = 1;
  h.steps = d.fine_steps;
  h.tmp = I.tmp.p;
  return setup_forcing(I, d, s);
}

// Block cyclic reduction set-up of every strip at tau = dt (fine) and
// tau = DT / coarse_steps (coarse), in the order the solve consumes it.
pr_status factorize_dd2_instance(Instance& I, const double* coef_x, const double* coef_y,
                                 hipStream_t s) {
  const pr_problem_desc& d = I.d;
  const int nx = d.nx, ny = d.ny;
  if (d.coef_mode == PR_COEF_NODAL_LOG) {
    HIPOK(launch_faces_from_theta_2d(coef_x, nx, ny, I.ax.p, I.ay.p, s));
  } else {
    HIPOK(hipMemcpyAsync(I.ax.p, coef_x, I.ax.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPOK(hipMemcpyAsync(I.ay.p, coef_y, I.ay.n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  int Wmax = 16;
  for (auto& S : I.strips2) Wmax = std::max(Wmax, S.W);
  const long W2 = (long)Wmax * Wmax;
  const int nE0 = (ny + 1) / 2, n1 = ny / 2, nE1 = (n1 + 1) / 2;
  DBuf aug0, augL, D[2], B[2], C[2];
  HIPOK(aug0.alloc((size_t)nE0 * 2 * W2));
  if (n1 > 0) {
    HIPOK(augL.alloc((size_t)nE1 * 4 * W2));
    for (int q = 0; q < 2; q++) {
      HIPOK(D[q].alloc((size_t)n1 * W2));
      HIPOK(B[q].alloc((size_t)n1 * W2));
      HIPOK(C[q].alloc((size_t)n1 * W2));
    }
  }
  std::vector<std::unique_ptr<DArr<DD2Copy>>> keep_c;
  std::vector<std::unique_ptr<DArr<DD2Gemm>>> keep_g;
  auto store = [&](const std::vector<DD2Copy>& jobs, int W) -> pr_status {
    if (jobs.empty()) return PR_OK;
    keep_c.push_back(std::make_unique<DArr<DD2Copy>>());
    HIPOK(keep_c.back()->upload(jobs));
    HIPOK(launch_dd2_store(keep_c.back()->p, (int)jobs.size(), W, s));
    return PR_OK;
  };
  auto gemm = [&](const std::vector<DD2Gemm>& jobs, int W) -> pr_status {
    if (jobs.empty()) return PR_OK;
    keep_g.push_back(std::make_unique<DArr<DD2Gemm>>());
    HIPOK(keep_g.back()->upload(jobs));
    HIPOK(launch_dd2_gemm(keep_g.back()->p, (int)jobs.size(), W, s));
    return PR_OK;
  };
  const double hx = 1.0 / (nx + 1), hy = 1.0 / (ny + 1);
  for (int coarse = 0; coarse < 2; coarse++) {
    const double tau = coarse ? I.tauG : I.dt;
    double* pool = coarse ? I.pool2c.p : I.pool2f.p;
    double* bcp = coarse ? I.bc2c.p : I.bc2f.p;
    double* trip = coarse ? I.tri2c.p : I.tri2f.p;
    for (auto& S : I.strips2) {
      const int W = S.W;
      const long w2 = (long)W * W;
      DD2Geo g{I.ax.p, I.ay.p, I.rho2.p + (long)S.colour * (2 * nx + 1), nx, ny,
               S.col0, S.w, W, 0, tau / (hx * hx), tau / (hy * hy), tau * d.c};
      HIPOK(launch_dd2_bc(g, bcp + S.bc0, s));
      // level 0: LU and inverses of the eliminated rows, then the level-1 blocks
      HIPOK(launch_dd2_tri_inv(g, nE0, aug0.p, 2 * w2, trip + S.tri0, s));
      if (n1 == 0) continue;
      HIPOK(launch_dd2_scale0(g, bcp + S.bc0, aug0.p, 2 * w2, D[0].p, B[0].p, C[0].p, s));
      int cur = 0;
      for (int l = 1; (ny >> l) > 0; l++) {
        const int n = ny >> l, nE = (n + 1) / 2;
        double *Dc = D[cur].p, *Bc = B[cur].p, *Cc = C[cur].p;
        HIPOK(launch_dd2_aug(Dc, Bc, Cc, nE, W, augL.p, s));
        HIPOK(launch_dd2_gj(augL.p, 4 * w2, nE, W, 4 * W, s));
        std::vector<DD2Copy> jobs;
        for (int a = 0; a < n; a++) {
          if (a % 2 == 0) {
            const double* A = augL.p + (long)(a / 2) * 4 * w2;
            jobs.push_back(DD2Copy{A + W, pool + S.dinv[l][a], 4 * W, 0});
            if (S.m2[l][a] >= 0) jobs.push_back(DD2Copy{A + 2 * W, pool + S.m2[l][a], 4 * W, 0});
            if (S.m3[l][a] >= 0) jobs.push_back(DD2Copy{A + 3 * W, pool + S.m3[l][a], 4 * W, 0});
          } else {
            jobs.push_back(DD2Copy{Bc + a * w2, pool + S.bm[l][a], W, 0});
            if (S.cm[l][a] >= 0) jobs.push_back(DD2Copy{Cc + a * w2, pool + S.cm[l][a], W, 0});
          }
        }
        pr_status st = store(jobs, W);
        if (st != PR_OK) return st;
        const int nn = n / 2;
        if (nn == 0) break;
        // kept row a -> alive row (a - 1) / 2 of level l + 1:
        //   D' = D_a - B_a M3_{a-1} - C_a M2_{a+1}, B' = -B_a M2_{a-1}, C' = -C_a M3_{a+1}
        const int nxt = 1 - cur;
        std::vector<DD2Gemm> g1, g2;
        for (int a = 1; a < n; a += 2) {
          const long o = (long)((a - 1) / 2) * w2;
          const double* Em = augL.p + (long)((a - 1) / 2) * 4 * w2;
          g1.push_back(DD2Gemm{Bc + a * w2, Em + 3 * W, Dc + a * w2, D[nxt].p + o, W, 4 * W, W, W, -1.0});
          g1.push_back(DD2Gemm{Bc + a * w2, Em + 2 * W, nullptr, B[nxt].p + o, W, 4 * W, W, W, -1.0});
          if (a + 1 < n) {
            const double* Ep = augL.p + (long)((a + 1) / 2) * 4 * w2;
            g1.push_back(DD2Gemm{Cc + a * w2, Ep + 3 * W, nullptr, C[nxt].p + o, W, 4 * W, W, W, -1.0});
            g2.push_back(DD2Gemm{Cc + a * w2, Ep + 2 * W, D[nxt].p + o, D[nxt].p + o, W, 4 * W, W, W, -1.0});
          } else {
            HIPOK(launch_fill_zero(C[nxt].p + o, w2, s));
          }
        }
        st = gemm(g1, W);
        if (st != PR_OK) return st;
        st = gemm(g2, W);
        if (st != PR_OK) return st;
        cur = nxt;
      }
    }
  }
  HIPOK(hipStreamSynchronize(s));  // set-up buffers and job lists are released on return
  return PR_OK;
}

// One colour's substep (I - tau A_k) over the strips of colour k: fine or
// coarse factors; the slice-minor fine workspace or the single state in tmp.
pr_status dd2_substep(pr_problem_s* P, Instance& I, bool coarse, bool single, int colour,
                      hipStream_t s) {
  const double* pool = coarse ? I.pool2c.p : I.pool2f.p;
  const double* bc = coarse ? I.bc2c.p : I.bc2f.p;
  double* Z = single ? I.tmp.p : I.Zs.p;
  double* Y = single ? I.Y1.p : I.Ys.p;
  const int Npad = single ? 1 : I.Npad2;
  PhaseTimer pt(P, single ? PH_COARSE_X : PH_FINE, s);
  const double* tri = coarse ? I.tri2c.p : I.tri2f.p;
  for (const auto& ph : I.phases2[colour]) {
    const DD2Row* rows = I.rows2.p + ph.off;
    if (ph.mode == DD2_KUP0)
      HIPOK(launch_dd2_kup0(rows, ph.cnt, bc, Z, Y, I.d.nx, Npad, s));
    else if (ph.mode == DD2_TRI_APPLY || ph.mode == DD2_TRI_BACK)
      // the single state: one wave per row; all slices: one lane per (row, slice)
      HIPOK(launch_dd2_tri0(ph.mode == DD2_TRI_BACK, rows, ph.cnt, ph.wmax, single, tri, bc, Z, Y,
                            I.d.nx, Npad, s));
    else
      HIPOK(launch_dd2_solve(ph.mode, I.units2.p + ph.off, ph.cnt, pool, Z, Y, I.d.nx, Npad,
                             single, single ? ph.split1 : ph.split, ph.waves, s));
  }
  return PR_OK;
}

// Douglas-Rachford terms of a fine step (eq. DR_method): S_k = dt A_k U_n for
// colours k >= 1 from the step's input Z (slice-minor, Npad columns), and
// Z += sum_k S_k, so that the first colour solves U_n + dt (A - A_0) U_n
// (+ dt F); colour k >= 1 then solves its input minus S_k.
pr_status dd2_dr_terms(Instance& I, double* Z, double* S, int Npad, hipStream_t s) {
  const int nx = I.d.nx, ny = I.d.ny;
  const long n = (long)nx * ny * Npad;
  const double hx = 1.0 / (nx + 1), hy = 1.0 / (ny + 1);
  for (int k = 1; k < I.n_colors; k++) {
    DD2Geo g{I.ax.p, I.ay.p, I.rho2.p + (long)k * (2 * nx + 1), nx, ny, 0, 0, 0, 0,
             I.dt / (hx * hx), I.dt / (hy * hy), I.dt * I.d.c};
    HIPOK(launch_dd2_stencil(g, Z, S + (k - 1) * n, Npad, s));
  }
  for (int k = 1; k < I.n_colors; k++) HIPOK(launch_dd2_axpy(Z, S + (k - 1) * n, 1.0, n, s));
  return PR_OK;
}

// One step of the single state in tmp (source at table entry gidx): FIE, or the
// Douglas-Rachford fine step when the instance's fine propagator is DR.
pr_status dd2_step_single(pr_problem_s* P, int i, bool coarse, long gidx, hipStream_t s) {
  Instance& I = *P->inst[i];
  const bool dr = !coarse && I.d.fine == PR_DR && I.n_colors > 1;
  const long n = I.npts;
  if (dr) {
    PhaseTimer pt(P, PH_OTHER, s);
    pr_status st = dd2_dr_terms(I, I.tmp.p, I.drS1.p, 1, s);
    if (st != PR_OK) return st;
  }
  if (I.h.nforce) {
    const long stride = coarse ? (long)I.d.n_slices * I.d.coarse_steps
                               : (long)I.d.n_slices * I.d.fine_steps;
    HIPOK(launch_force_state(P->d_inst + i, I.h, I.tmp.p, coarse ? I.fgc.p : I.fgf.p, gidx, stride,
                             s));
  }
  for (int k = 0; k < I.n_colors; k++) {
    if (dr && k > 0) HIPOK(launch_dd2_axpy(I.tmp.p, I.drS1.p + (k - 1) * n, -1.0, n, s));
    pr_status st = dd2_substep(P, I, coarse, true, k, s);
    if (st != PR_OK) return st;
  }
  return PR_OK;
}

// Fine propagation of every slice of a 2D DD instance: slice-minor workspace,
// fine steps with the source on the first substep, back to slices.
pr_status dd2_fine(pr_problem_s* P, Instance& I, const double* U, double* out, hipStream_t s) {
  const long npts = I.npts;
  const int N = I.d.n_slices, Np = I.Npad2;
  {
    PhaseTimer pt(P, PH_TRANSPOSE, s);
    HIPOK(launch_dd2_to_sm(U, I.Zs.p, npts, N, Np, s));
  }
  const bool dr = I.d.fine == PR_DR && I.n_colors > 1;
  const long n = npts * Np;
  for (int t = 0; t < I.d.fine_steps; t++) {
    if (dr) {
      PhaseTimer pt(P, PH_OTHER, s);
      pr_status st = dd2_dr_terms(I, I.Zs.p, I.drS2.p, Np, s);
      if (st != PR_OK) return st;
    }
    if (I.h.nforce) {
      PhaseTimer pt(P, PH_OTHER, s);
      HIPOK(launch_dd2_force_sm(I.fS.p, I.fgf.p, (long)N * I.d.fine_steps, I.d.fine_steps, t,
                                I.Zs.p, npts, N, Np, s));
    }
    for (int k = 0; k < I.n_colors; k++) {
      if (dr && k > 0) {
        PhaseTimer pt(P, PH_OTHER, s);
        HIPOK(launch_dd2_axpy(I.Zs.p, I.drS2.p + (k - 1) * n, -1.0, n, s));
      }
      pr_status st = dd2_substep(P, I, false, false, k, s);
      if (st != PR_OK) return st;
    }
  }
  PhaseTimer pt(P, PH_TRANSPOSE, s);
  HIPOK(launch_dd2_from_sm(I.Zs.p, out, npts, N, Np, s));
  return PR_OK;
}

// Work list of one direction for the instances in `members` (all-slices
// variant): items (inst, b, group), ordered so that line groups whose values
// share the previous sweep's chunk carries run on the same XCD (workgroups are
// dealt to the 8 XCDs round-robin by id).
std::vector<WorkItem> build_work(const std::vector<int>& members,
                                 const std::vector<std::unique_ptr<Instance>>& inst, int dir,
                                 int M, int b_lo = 0, int b_hi = 1 << 30, int per_item = 1) {
  const int kXcd = 8;
  std::vector<std::vector<WorkItem>> per(kXcd);
  for (int m : members) {
    const DimInst& h = inst[m]->h;
    if (dir == 1 && inst[m]->d.dim == 1) continue;
    const int n_lines = dir == 0 ? h.ny : h.nx;
    const int G = 64 / h.L * per_item;  // lines per work item
    const int n_groups = (n_lines + G - 1) / G;
    const int groups_per_chunk = std::max(1, M / G);
    for (int b = std::max(0, b_lo); b < std::min(h.B, b_hi); b++)
      for (int g = 0; g < n_groups; g++) {
        int x = (g / groups_per_chunk) % kXcd;
        per[x].push_back(WorkItem{m, b, g, 0});
      }
  }
  std::vector<WorkItem> out;
  size_t longest = 0;
  for (auto& v : per) longest = std::max(longest, v.size());
  for (size_t r = 0; r < longest; r++)
    for (int x = 0; x < kXcd; x++)
      if (r < per[x].size()) out.push_back(per[x][r]);
  return out;
}

// Appends `items` to `out` in launch order such that, with workgroups dealt to
// the 8 XCDs round-robin, each XCD receives a contiguous range of the list
// (neighbouring line blocks share cache lines).
template <typename Item>
void append_xcd_ordered(const std::vector<Item>& items, std::vector<Item>& out) {
  const int nb = (int)items.size(), per = nb / 8, rem = nb % 8;
  for (int bid = 0; bid < nb; bid++) {
    const int x = bid % 8, r = bid / 8;
    out.push_back(items[x * per + std::min(x, rem) + r]);
  }
}

hipError_t upload_work(const std::vector<WorkItem>& w, WorkItem** d, int* n) {
  *n = (int)w.size();
  if (w.empty()) return hipSuccess;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(d), w.size() * sizeof(WorkItem));
  if (e != hipSuccess) return e;
  return hipMemcpy(*d, w.data(), w.size() * sizeof(WorkItem), hipMemcpyHostToDevice);
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Fine propagation of every slice of every instance: in_base + per-instance
// offset (slices or states layout) -> out_base + slices offset.
pr_status fine_all(pr_problem_s* P, const double* in_base, bool in_states_layout, double* out_base,
                   hipStream_t s, const std::vector<char>* host_active = nullptr) {
  const int n = (int)P->inst.size();
  // domain-decomposition instances that have converged are skipped on the host
  // (the dimensional kernels read the device mask themselves)
  auto skip = [&](int i) { return P->inst[i]->dd && host_active && !(*host_active)[i]; };
  for (int i = 0; i < n; i++) {
    Instance& I = *P->inst[i];
    const double* U = in_base + (in_states_layout ? I.off_states : I.off_slices);
    if (skip(i)) continue;
    if (I.dd2) {
      pr_status st = dd2_fine(P, I, U, out_base + I.off_slices, s);
      if (st != PR_OK) return st;
      continue;
    }
    PhaseTimer pt(P, PH_TRANSPOSE, s);
    HIPOK(launch_to_interleaved(P->d_inst + i, I.h, U, s, I.part));
  }
  // all instances advance step by step; one grouped launch per lane width and
  // direction (per pass of slice blocks when passes are enabled: a pass runs all
  // its steps before the next one starts, keeping its working set cached)
  int smax = 0;
  for (auto& I : P->inst) smax = std::max(smax, I->d.fine_steps);
  {
    PhaseSpan sp(P, PH_FINE, s);
    for (int q = 0; q < P->n_passes; q++) {
      for (int t = 0; t < smax; t++) {
        for (auto& g : P->groups) {
          if (g.dr && t == 0) {  // S = dt A_y U of the input; later steps' S come from the y sweep
            PhaseTimer pt(P, PH_FINE, s);
            for (int i : g.members)
              HIPOK(launch_dr_stencil(P->d_inst + i, P->inst[i]->h, 0, t, q * P->pass_blocks,
                                      (q + 1) * P->pass_blocks, s));
            sp.add();
          }
          if (g.part) {  // all slice blocks in the first pass
            if (q > 0) continue;
            for (int dir = 0; dir < 2; dir++) {
              PhaseTimer pt(P, PH_FINE, s);
              HIPOK(launch_part_sweep(P->d_inst, g.d_pwork[dir], g.n_pwork[dir], dir, t,
                                      g.pwaves[dir], g.ppl[dir], dir == 0 && g.ft, s));
              sp.add();
            }
            continue;
          }
          for (int dir = 0; dir < 2; dir++) {
            const int off = g.pass_off[dir][q], cnt = g.pass_off[dir][q + 1] - off;
            if (!cnt) continue;
            PhaseTimer pt(P, PH_FINE, s);
            HIPOK(launch_fine_sweep(P->d_inst, g.d_work[dir] + off, cnt, g.L, g.M, dir,
                                    dir == 1 || t > 0, t, s, g.dr ? (dir == 0 ? 1 : -1) : 0,
                                    dir == 0 && g.ft, P->twisted, g.grouped, g.long_lines));
            sp.add();
          }
        }
      }
    }
  }
  for (int i = 0; i < n; i++) {
    Instance& I = *P->inst[i];
    if (!I.dd || I.dd2 || skip(i)) continue;
    PhaseSpan sp(P, PH_FINE, s);
    for (int t = 0; t < I.d.fine_steps; t++) {
      if (I.h.nforce) {
        PhaseTimer pt(P, PH_FINE, s);
        HIPOK(launch_force_interleaved(P->d_inst + i, I.h, t, s));
        sp.add();
      }
      pr_status st = dd_fie_step(P, I, false, 0, t, s);
      if (st != PR_OK) return st;
      sp.add(I.n_colors);  // one colour substep per colour
    }
  }
  for (int i = 0; i < n; i++) {
    Instance& I = *P->inst[i];
    if (I.dd2 || skip(i)) continue;
    PhaseTimer pt(P, PH_TRANSPOSE, s);
    if (I.dd)
      HIPOK(launch_dd_from_interleaved(I.d_dd, I.hdd, I.ffine.view(), out_base + I.off_slices, s));
    else
      HIPOK(launch_from_interleaved(P->d_inst + i, I.h, out_base + I.off_slices, !I.part, s,
                                    I.part));
  }
  return PR_OK;
}

// One coarse propagation G (coarse_steps FIE steps) of state src of DD
// instance i, followed by the parareal update in `mode` (see launch_update).
pr_status coarse_apply_dd(pr_problem_s* P, int i, int n, const double* src, int mode,
                          const double* F, double* Gold, double* Unext, hipStream_t s) {
  Instance& I = *P->inst[i];
  HIPOK(launch_copy(src, I.tmp.p, I.npts, s));
  const int cs = I.d.coarse_steps;
  for (int c = 0; c < cs; c++) {
    if (I.dd2) {
      pr_status st = dd2_step_single(P, i, true, (long)n * cs + c, s);
      if (st != PR_OK) return st;
      continue;
    }
    if (I.h.nforce)
      HIPOK(launch_force_state(P->d_inst + i, I.h, I.tmp.p, I.fgc.p, (long)n * cs + c,
                               (long)I.d.n_slices * cs, s));
    pr_status st = dd_fie_step(P, I, true, 1, 0, s);
    if (st != PR_OK) return st;
  }
  PhaseTimer pt(P, PH_COARSE_Y, s);
  HIPOK(launch_update(I.tmp.p, F, Gold, Unext, I.npts, mode, I.h.incp, s));
  return PR_OK;
}

// Coarse sweep of every instance. Dimensional instances: one batched x and
// one batched y launch per (slice index, coarse step) over all instances that
// have that slice and are active on the device. DD instances: per instance,
// skipped when host_active says so.
pr_status coarse_sweep_impl(pr_problem_s* P, const double* F, double* Gold, double* U,
                            unsigned long long* inc_bits, hipStream_t s,
                            const std::vector<char>* host_active) {
  const int n = (int)P->inst.size();
  unsigned long long* inc = inc_bits ? inc_bits : P->d_inc;
  HIPOK(launch_fill_zero(reinterpret_cast<double*>(inc), n, s));
  HIPOK(launch_fill_zero(reinterpret_cast<double*>(P->d_incp), P->n_incp, s));
  for (int i = 0; i < n; i++) {
    Instance& I = *P->inst[i];
    if (!I.dd || (host_active && !(*host_active)[i])) continue;
    PhaseSpan sp(P, PH_COARSE, s);
    for (int k = 0; k < I.d.n_slices; k++) {
      const double* Un = U + I.off_states + (size_t)k * I.npts;
      double* Unext = U + I.off_states + (size_t)(k + 1) * I.npts;
      double* Gk = Gold + I.off_slices + (size_t)k * I.npts;
      const double* Fk = F ? F + I.off_slices + (size_t)k * I.npts : nullptr;
      pr_status st = coarse_apply_dd(P, i, k, Un, F ? 1 : 2, Fk, Gk, Unext, s);
      if (st != PR_OK) return st;
      sp.add();  // one coarse step of one slice
    }
  }
  bool segx = false, segy = false;
  for (auto& I : P->inst)
    if (!I->dd) {
      segx = segx || I->h.Sx > 1;
      segy = segy || I->h.Sy > 1;
    }
  PhaseSpan sp(P, PH_COARSE, s);
  for (int k = 0; k < P->Nmax; k++) {
    const int xb = P->xoff[k], xn = P->xoff[k + 1] - xb;
    const int yb = P->yoff[k], yn = P->yoff[k + 1] - yb;
    if (xn == 0 && yn == 0) continue;
    for (int c = 0; c < P->csmax; c++) {
      {
        PhaseTimer pt(P, PH_COARSE_X, s);
        HIPOK(launch_coarse_xb(P->d_inst, P->xitems.p + xb, xn, k, c, U, s, segx));
      }
      PhaseTimer pt(P, PH_COARSE_Y, s);
      HIPOK(launch_coarse_yb(P->d_inst, P->yitems.p + yb, yn, k, c, F ? 1 : 2, F, Gold, U, s,
                             segy));
      sp.add(2);
    }
  }
  HIPOK(launch_inc_reduce(P->d_inst, n, inc, s));
  return PR_OK;
}

pr_status seq_fine_dim(pr_problem_s* p, int i, const double* u0, double* U, hipStream_t s) {
  {
    Instance& I = *p->inst[i];
    const DimInst* dI = p->d_inst + i;
    if (U != u0) HIPOK(launch_copy(u0, U, I.npts, s));
    for (int k = 0; k < I.d.n_slices; k++) {
      const double* src = U + (size_t)k * I.npts;
      double* dst = U + (size_t)(k + 1) * I.npts;
      for (int t = 0; t < I.d.fine_steps; t++) {
        const double* in = t == 0 ? src : I.tmp.p;
        const bool last = t + 1 == I.d.fine_steps;
        // source at the end of fine step t of slice k
        const double* gtab = I.h.nforce ? I.fgf.p : nullptr;
        const long gidx = (long)k * I.d.fine_steps + t;
        const long gstride = (long)I.d.n_slices * I.d.fine_steps;
        if (I.h.dr) {
          // S = dt A_y U into drS[0, npts), U + S into drS[npts, 2 npts); x solve;
          // subtract S; y solve
          double* UpS = I.drS.p + I.npts;
          {
            PhaseTimer pt(p, PH_COARSE_X, s);
            HIPOK(launch_dr_stencil_nat(dI, I.h, in, UpS, 0, s));
            HIPOK(launch_coarse_x(dI, I.h, UpS, I.tmp.p, true, s, gtab, gidx, gstride));
            HIPOK(launch_dr_stencil_nat(dI, I.h, nullptr, I.tmp.p, 1, s));
          }
          PhaseTimer pt(p, PH_COARSE_Y, s);
          HIPOK(launch_coarse_y(dI, I.h, I.tmp.p, last ? dst : I.tmp.p, true, s));
          continue;
        }
        {
          PhaseTimer pt(p, PH_COARSE_X, s);
          HIPOK(launch_coarse_x(dI, I.h, in, I.tmp.p, true, s, gtab, gidx, gstride));
        }
        PhaseTimer pt(p, PH_COARSE_Y, s);
        HIPOK(launch_coarse_y(dI, I.h, I.tmp.p, last ? dst : I.tmp.p, true, s));
      }
    }
  }
  return PR_OK;
}

pr_status set_all_active(pr_problem_s* P, hipStream_t s) {
  std::vector<int> ones(P->inst.size(), 1);
  HIPOK(hipMemcpyAsync(P->d_active, ones.data(), ones.size() * sizeof(int), hipMemcpyHostToDevice,
                       s));
  HIPOK(hipStreamSynchronize(s));
  return PR_OK;
}

// Device descriptors, grouped fine-sweep work lists (by lane width) and the
// per-slice-index item lists of the batched coarse sweeps.
pr_status build_schedules(pr_problem_s* P) {
  const int n = (int)P->inst.size();
  // partitioned sweeps: 2D FIE instances whose lines fit one workgroup in both
  // directions with the instance's fullest slice block
  for (auto& Ip : P->inst) {
    Instance& I = *Ip;
    I.part = false;
    if (I.dd) continue;
    DimInst& h = I.h;
    const bool on = I.plx0 > 0 && I.ply0 > 0 &&
                    (P->part_sweeps == 2 || (P->part_sweeps == 1 && h.N <= kPartMaxSlices));
    h.plx = on ? I.plx0 : 0;
    h.ply = on ? I.ply0 : 0;
  }
  std::vector<DimInst> hd(n);
  for (int i = 0; i < n; i++) hd[i] = P->inst[i]->h;
  HIPOK(hipMemcpy(P->d_inst, hd.data(), hd.size() * sizeof(DimInst), hipMemcpyHostToDevice));
  for (auto& g : P->groups) {
    for (auto*& w : g.d_work)
      if (w) {
        (void)hipFree(w);
        w = nullptr;
      }
    for (auto*& w : g.d_pwork)
      if (w) {
        (void)hipFree(w);
        w = nullptr;
      }
  }
  P->groups.clear();
  int Bmax = 1;
  for (auto& I : P->inst)
    if (!I->dd) Bmax = std::max(Bmax, I->h.B);
  const int bpp = P->blocks_per_pass > 0 ? P->blocks_per_pass : Bmax;
  P->n_passes = (Bmax + bpp - 1) / bpp;
  P->pass_blocks = bpp;
  for (int L = 1; L <= 64; L <<= 1)
    for (int key = 0; key < 8; key++) {
      const int dr = key & 1, ft = (key >> 1) & 1, pt = key >> 2;
      std::vector<int> members;
      for (int i = 0; i < n; i++) {
        const DimInst& hi = P->inst[i]->h;
        if (!P->inst[i]->dd && hi.L == L && hi.dr == dr && (hi.nforce > 0) == (ft == 1) &&
            (hi.plx > 0 && hi.ply > 0) == (pt == 1))
          members.push_back(i);
      }
      if (members.empty()) continue;
      pr_problem_s::Group g;
      g.L = L;
      g.dr = dr;
      g.ft = ft;
      g.M = dr ? kDRChunk : P->M;
      g.grouped = L == 64 && !dr && P->twisted && P->grouped && (g.M == 20 || g.M == 24);
      g.members = members;
      for (int i : members) {
        const DimInst& hi = P->inst[i]->h;
        if (std::max(hi.Px, hi.Py) > lds_chunk_lines(g.M)) g.long_lines = true;
      }
      for (int dir = 0; dir < 2; dir++) {
        std::vector<WorkItem> all;
        g.pass_off[dir].assign(1, 0);
        for (int q = 0; q < P->n_passes; q++) {
          std::vector<WorkItem> part = build_work(members, P->inst, dir, g.M, q * bpp, (q + 1) * bpp,
                                                  g.grouped ? grouped_lines() : 1);
          all.insert(all.end(), part.begin(), part.end());
          g.pass_off[dir].push_back((int)all.size());
        }
        HIPOK(upload_work(all, &g.d_work[dir], &g.n_work[dir]));
      }
      g.part = pt == 1;  // every member's lines fit a workgroup
      if (g.part) {
        for (int dir = 0; dir < 2; dir++) {
          std::vector<WorkItem> items;
          for (int i : members) {
            const DimInst& hi = P->inst[i]->h;
            const int n_lines = dir == 0 ? hi.ny : hi.nx, n_pos = dir == 0 ? hi.nx : hi.ny;
            const int Pl = dir == 0 ? hi.plx : hi.ply;
            g.pwaves[dir] = std::max(g.pwaves[dir], part_waves(n_pos, Pl, hi.Lp));
            g.ppl[dir] = std::max(g.ppl[dir], Pl);
            // the blocks of a line share its factor rows, neighbouring y-lines
            // the cache lines of their nodes
            for (int ln = 0; ln < n_lines; ln++)
              for (int b = 0; b < hi.Bp; b++) items.push_back(WorkItem{i, b, ln, 0});
          }
          std::vector<WorkItem> ordered;
          append_xcd_ordered(items, ordered);
          HIPOK(upload_work(ordered, &g.d_pwork[dir], &g.n_pwork[dir]));
        }
        for (int i : members) P->inst[i]->part = true;
      }
      P->groups.push_back(g);
    }
  P->Nmax = 0;
  P->csmax = 0;
  P->max_nx = 1;
  P->max_ny = 1;
  P->any_dd = false;
  for (auto& I : P->inst) {
    if (I->dd) {
      P->any_dd = true;
      continue;
    }
    P->Nmax = std::max(P->Nmax, I->d.n_slices);
    P->csmax = std::max(P->csmax, I->d.coarse_steps);
    P->max_nx = std::max(P->max_nx, I->d.nx);
    P->max_ny = std::max(P->max_ny, I->d.ny);
  }
  std::vector<LineItem> xi, yi;
  P->xoff.assign(1, 0);
  P->yoff.assign(1, 0);
  for (int k = 0; k < P->Nmax; k++) {
    std::vector<LineItem> xk, yk;
    for (int i = 0; i < n; i++) {
      const Instance& I = *P->inst[i];
      if (I.dd || I.d.n_slices <= k) continue;
      for (int rb = 0; rb < (I.d.ny + kCoarseRowsPerBlock - 1) / kCoarseRowsPerBlock; rb++)
        xk.push_back(LineItem{i, rb});
      for (int cb = 0; cb < (I.d.nx + kCoarseColsPerBlock - 1) / kCoarseColsPerBlock; cb++)
        yk.push_back(LineItem{i, cb});
    }
    append_xcd_ordered(xk, xi);
    append_xcd_ordered(yk, yi);
    P->xoff.push_back((int)xi.size());
    P->yoff.push_back((int)yi.size());
  }
  HIPOK(P->xitems.upload(xi));
  HIPOK(P->yitems.upload(yi));
  return PR_OK;
}

// Lane width (lines per wave = 64 / L) and chunk length of the fine sweeps.
// lanes_cap = 0 keeps every instance's default L; otherwise L = min(cap, default).
// Workspaces were sized for the default L and M = 16, which bound every choice.
pr_status apply_layout(pr_problem_s* P, int lanes_cap, int M, bool twisted) {
  HIPOK(hipDeviceSynchronize());
  for (auto& Ip : P->inst) {
    Instance& I = *Ip;
    if (I.dd) continue;
    DimInst& h = I.h;
    const int nx = I.d.nx, ny = I.d.ny, N = I.d.n_slices;
    const int L = lanes_cap ? std::min(lanes_cap, I.Ldef) : I.Ldef;
    h.L = L;
    h.B = (N + L - 1) / L;
    h.slab = (long)nx * ny * L;
    const int Mi = I.d.fine == PR_DR ? kDRChunk : M;
    const int Mprev = h.M, twx = h.twx, twy = h.twy;
    h.M = Mi;
    h.Px = (nx + Mi - 1) / Mi;
    h.Py = (ny + Mi - 1) / Mi;
    set_twist(h, twisted);
    if (h.M != Mprev || h.twx != twx || h.twy != twy) {
      pr_status st = fine_factors(I, nullptr);
      if (st != PR_OK) return st;
    }
  }
  P->M = M;
  P->twisted = twisted;
  P->lanes_cap = lanes_cap;
  HIPOK(hipDeviceSynchronize());
  if (P->gexec) {
    (void)hipGraphExecDestroy(P->gexec);
    P->gexec = nullptr;
  }
  if (P->graph) {
    (void)hipGraphDestroy(P->graph);
    P->graph = nullptr;
  }
  return build_schedules(P);
}


// ------------------------------------------------------ serial adjoint ---
// Workspace of the serial adjoint: the post-x (W) and post-y (V) states of
// every fine step of one slice, lambda, mu, the face-gradient accumulators and
// the slice-boundary checkpoints.
struct AdjWork {
  double *W, *V, *lam, *mu, *gax, *gay, *ckpt;
};

pr_status check_adjoint_args(pr_problem_s* p, const double* u0, const double* lambda_T,
                             const double* grad_u0, const double* grad_coef, const char* who) {
  if (!p || !u0 || !lambda_T || !grad_u0 || !grad_coef) return fail(PR_EINVAL, "NULL argument");
  if (p->inst.size() != 1) return fail(PR_EUNSUPPORTED, "%s needs a single-instance handle", who);
  const Instance& I = *p->inst[0];
  if (I.dd || I.d.dim != 2)
    return fail(PR_EUNSUPPORTED, "%s supports 2D dimensional splitting", who);
  if (I.d.fine != PR_FIE)
    return fail(PR_EUNSUPPORTED, "%s supports the FIE fine propagator only", who);
  return PR_OK;
}

// Adjoint of the fine map (transpose of eq. FIE_method, in reverse substep
// order): forward checkpoints at the slice boundaries, then per slice in
// reverse the recompute of its W and V states and its reverse steps, each
// followed by the face-gradient accumulation; the theta chain rule (or a copy
// of the face gradients) at the end. Every part of w is written before it is
// read; the accumulators are cleared here.
pr_status adjoint_serial(pr_problem_s* p, const double* u0, const double* lambda_T,
                         double* grad_u0, double* grad_coef, const AdjWork& w, hipStream_t s) {
  Instance& I = *p->inst[0];
  const int nx = I.d.nx, ny = I.d.ny, N = I.d.n_slices, S = I.d.fine_steps;
  const size_t npts = I.npts;
  const size_t ngx = (size_t)ny * (nx + 1), ngy = (size_t)(ny + 1) * nx;
  const DimInst* dI = p->d_inst;
  pr_status st = seq_fine_dim(p, 0, u0, w.ckpt, s);
  if (st != PR_OK) return st;
  HIPOK(launch_fill_zero(w.gax, ngx, s));
  HIPOK(launch_fill_zero(w.gay, ngy, s));
  HIPOK(launch_copy(lambda_T, w.lam, npts, s));
  const double hx = 1.0 / (nx + 1), hy = 1.0 / (ny + 1);
  const double cx = I.dt / (hx * hx), cy = I.dt / (hy * hy);
  for (int n = N - 1; n >= 0; n--) {
    // recompute the slice's fine steps from its checkpoint
    for (int t = 0; t < S; t++) {
      const double* prev = t == 0 ? w.ckpt + (size_t)n * npts : w.V + (size_t)(t - 1) * npts;
      {
        PhaseTimer pt(p, PH_COARSE_X, s);
        HIPOK(launch_coarse_x(dI, I.h, prev, w.W + (size_t)t * npts, true, s,
                              I.h.nforce ? I.fgf.p : nullptr, (long)n * S + t, (long)N * S));
      }
      PhaseTimer pt(p, PH_COARSE_Y, s);
      HIPOK(launch_coarse_y(dI, I.h, w.W + (size_t)t * npts, w.V + (size_t)t * npts, true, s));
    }
    // reverse the steps: transposed (= same, symmetric) solves in reverse substep order
    for (int t = S - 1; t >= 0; t--) {
      {
        PhaseTimer pt(p, PH_COARSE_Y, s);
        HIPOK(launch_coarse_y(dI, I.h, w.lam, w.mu, true, s));
      }
      HIPOK(launch_face_grad_y(w.mu, w.V + (size_t)t * npts, nx, ny, cy, w.gay, s));
      {
        PhaseTimer pt(p, PH_COARSE_X, s);
        HIPOK(launch_coarse_x(dI, I.h, w.mu, w.lam, true, s));
      }
      HIPOK(launch_face_grad_x(w.lam, w.W + (size_t)t * npts, nx, ny, cx, w.gax, s));
    }
  }
  HIPOK(launch_copy(w.lam, grad_u0, npts, s));
  if (I.d.coef_mode == PR_COEF_NODAL_LOG) {
    HIPOK(launch_theta_chain(I.theta.p, w.gax, w.gay, nx, ny, grad_coef, s));
  } else {
    HIPOK(launch_copy(w.gax, grad_coef, ngx, s));
    HIPOK(launch_copy(w.gay, grad_coef + ngx, ngy, s));
  }
  return PR_OK;
}

// --------------------------------------------- allocation-free scratch ---
// pr_adjoint_noalloc keeps its workspace in this file-scope device array
// instead of allocating: every GPU the library runs on holds one copy (in the
// library's code object) until the process ends. In host code the name is
// only a stand-in: its device address, per GPU, comes from
// hipGetSymbolAddress, taken once per device with that device current (by
// pr_create_problem, or by the entry point's first call on a device), and
// only that address is handed to kernels.
constexpr size_t kNoAllocScratchDoubles = size_t(8) << 20;  // 64 MiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch array.
pr_status device_scratch(double** out) {
  int dev = 0;
  HIPOK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PR_EUNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPOK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(PR_EDEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return PR_OK;
}

}  // namespace

extern "C" {

const char* pr_last_error(void) { return g_err; }

pr_status pr_profile_control(pr_problem p, int mode) {
  return guarded([&]() -> pr_status {
    if (!p) return fail(PR_EINVAL, "NULL handle");
    if (mode == 0 || mode == 1 || mode == 3) {
      p->prof = mode != 0;
      p->prof_span = mode == 3;
    } else if (mode == 2) {
      pr_profile z{};
      p->acc = z;
      HIPOK(hipDeviceSynchronize());
      for (auto& r : p->recs) {
        p->ev_free.push_back(r.a);
        p->ev_free.push_back(r.b);
      }
      p->recs.clear();
    } else {
      return fail(PR_EINVAL, "mode must be 0, 1, 2 or 3");
    }
    return PR_OK;
  });
}

pr_status pr_profile_read(pr_problem p, pr_profile* out) {
  return guarded([&]() -> pr_status {
    if (!p || !out) return fail(PR_EINVAL, "NULL argument");
    for (auto& r : p->recs) {
      HIPOK(hipEventSynchronize(r.b));
      float ms = 0.f;
      HIPOK(hipEventElapsedTime(&ms, r.a, r.b));
      p->acc.ms[r.phase] += ms;
      p->acc.count[r.phase] += r.n;
      p->ev_free.push_back(r.a);
      p->ev_free.push_back(r.b);
    }
    p->recs.clear();
    *out = p->acc;
    return PR_OK;
  });
}

pr_status pr_create_problem(const pr_problem_desc* descs, int n_instances, void* hip_stream,
                            pr_problem* out) {
  return guarded([&]() -> pr_status {
    if (!out) return fail(PR_EINVAL, "out is NULL");
    *out = nullptr;
    if (!descs || n_instances < 1) return fail(PR_EINVAL, "need at least one descriptor");
    for (int i = 0; i < n_instances; i++) {
      pr_status st = validate(descs[i], i);
      if (st != PR_OK) return st;
    }
    hipStream_t s = as_stream(hip_stream);
    {  // device address of this GPU's allocation-free scratch (pr_adjoint_noalloc)
      double* scr = nullptr;
      pr_status st = device_scratch(&scr);
      if (st != PR_OK) return st;
    }
    std::unique_ptr<pr_problem_s> P(new (std::nothrow) pr_problem_s());
    if (!P) return fail(PR_ENOMEM, "host allocation failed");
    // Default fine-sweep form: one wave per (line group, slice block) gives
    // `waves` waves per sweep; below two per SIMD of the chip the lines are
    // twisted (two waves each, short chunks, grouped carries), otherwise one
    // wave per line with long chunks keeps the per-wave overheads lowest.
    // Twisted 64-slice FIE lines run grouped, whose loads are balanced at chunk
    // 20; the other forms keep the long chunk.
    {
      long waves = 0;
      bool any_grouped = false;
      for (int i = 0; i < n_instances; i++) {
        const pr_problem_desc& d = descs[i];
        if (d.split != PR_SPLIT_DIM) continue;
        const int L = std::min(64, std::max(8, pow2_at_least(d.n_slices)));
        const long B = (d.n_slices + L - 1) / L, G = 64 / L;
        waves += B * std::max((d.ny + G - 1) / G, (d.nx + G - 1) / G);
        any_grouped = any_grouped || (L == 64 && d.fine == PR_FIE);
      }
      P->twisted = waves < kTwistBelowWaves;
      P->M = P->twisted && any_grouped ? 20 : 32;
    }
    size_t ou = 0, osl = 0, ost = 0;
    for (int i = 0; i < n_instances; i++) {
      auto I = std::make_unique<Instance>();
      I->d = descs[i];
      I->d.coef_x = I->d.coef_y = I->d.rho = nullptr;
      const size_t npts = (size_t)descs[i].nx * descs[i].ny;
      I->off_u0 = ou; I->off_slices = osl; I->off_states = ost;
      ou += npts; osl += npts * descs[i].n_slices; ost += npts * (descs[i].n_slices + 1);
      pr_status st;
      if (descs[i].split == PR_SPLIT_DD && descs[i].dim == 2) {
        st = setup_dd2_instance(*I, descs[i].rho, s);
        if (st != PR_OK) return st;
        st = factorize_dd2_instance(*I, descs[i].coef_x, descs[i].coef_y, s);
      } else if (descs[i].split == PR_SPLIT_DD) {
        st = setup_dd_instance(P.get(), *I, descs[i].rho, s);
        if (st != PR_OK) return st;
        st = factorize_dd_instance(*I, descs[i].coef_x, s);
      } else {
        st = setup_dim_instance(P.get(), *I, s);
        if (st != PR_OK) return st;
        st = factorize_instance(P.get(), *I, descs[i].coef_x, descs[i].coef_y, s);
      }
      if (st != PR_OK) return st;
      P->inst.push_back(std::move(I));
    }
    P->tot_u0 = ou; P->tot_slices = osl; P->tot_states = ost;
    HIPOK(hipMalloc(reinterpret_cast<void**>(&P->d_active), n_instances * sizeof(int)));
    HIPOK(hipMalloc(reinterpret_cast<void**>(&P->d_inst), n_instances * sizeof(DimInst)));
    for (int i = 0; i < n_instances; i++) {
      DimInst& h = P->inst[i]->h;
      h.idx = i;
      h.cs = P->inst[i]->d.coarse_steps;
      h.npts = P->inst[i]->npts;
      h.off_slices = (long)P->inst[i]->off_slices;
      h.off_states = (long)P->inst[i]->off_states;
      h.active = P->d_active;
    }
    // per-block increment maxima of the coarse sweeps: one per column block of
    // the batched y launches, one per block of the DD update kernel
    for (auto& I : P->inst) {
      I->h.n_incp = I->dd ? update_blocks(I->npts)
                          : (I->d.nx + kCoarseColsPerBlock - 1) / kCoarseColsPerBlock;
      P->n_incp += I->h.n_incp;
    }
    HIPOK(hipMalloc(reinterpret_cast<void**>(&P->d_incp), P->n_incp * sizeof(unsigned long long)));
    {
      size_t o = 0;
      for (auto& I : P->inst) {
        I->h.incp = P->d_incp + o;
        o += I->h.n_incp;
      }
    }
    {
      pr_status st = set_all_active(P.get(), s);
      if (st != PR_OK) return st;
      st = build_schedules(P.get());
      if (st != PR_OK) return st;
    }
    HIPOK(hipStreamCreateWithFlags(&P->gstream, hipStreamNonBlocking));
    // parareal workspace
    HIPOK(P->F.alloc(osl));
    HIPOK(P->Gold.alloc(osl));
    HIPOK(hipMalloc(reinterpret_cast<void**>(&P->d_inc), n_instances * sizeof(unsigned long long)));
    HIPOK(hipHostMalloc(reinterpret_cast<void**>(&P->h_inc), n_instances * sizeof(double)));
    HIPOK(hipStreamSynchronize(s));
    *out = P.release();
    return PR_OK;
  });
}

pr_status pr_destroy_problem(pr_problem p) {
  return guarded([&]() -> pr_status {
    if (!p) return PR_OK;
    (void)hipDeviceSynchronize();
    delete p;
    return PR_OK;
  });
}

pr_status pr_num_instances(pr_problem p, int* n) {
  return guarded([&]() -> pr_status {
    if (!p || !n) return fail(PR_EINVAL, "NULL argument");
    *n = (int)p->inst.size();
    return PR_OK;
  });
}

pr_status pr_query_layout(pr_problem p, pr_instance_layout* per, size_t* totals) {
  return guarded([&]() -> pr_status {
    if (!p) return fail(PR_EINVAL, "NULL handle");
    if (per)
      for (size_t i = 0; i < p->inst.size(); i++) {
        const Instance& I = *p->inst[i];
        per[i].u0_offset = I.off_u0;
        per[i].slices_offset = I.off_slices;
        per[i].states_offset = I.off_states;
        per[i].npts = I.npts;
        per[i].n_slices = I.d.n_slices;
      }
    if (totals) {
      totals[0] = p->tot_u0;
      totals[1] = p->tot_slices;
      totals[2] = p->tot_states;
    }
    return PR_OK;
  });
}

pr_status pr_set_coefficients(pr_problem p, int instance, const double* coef_x,
                              const double* coef_y, void* hip_stream) {
  return guarded([&]() -> pr_status {
    if (!p) return fail(PR_EINVAL, "NULL handle");
    if (instance < 0 || instance >= (int)p->inst.size()) return fail(PR_EINVAL, "bad instance");
    Instance& I = *p->inst[instance];
    if (!coef_x || (I.d.dim == 2 && I.d.coef_mode == PR_COEF_FACES && !coef_y))
      return fail(PR_EINVAL, "NULL coefficient pointer");
    if (p->adjT) {  // the transposed problem of the parallel adjoint is rebuilt on demand
      (void)hipDeviceSynchronize();
      delete p->adjT;
      p->adjT = nullptr;
    }
    if (I.dd2) return factorize_dd2_instance(I, coef_x, coef_y, as_stream(hip_stream));
    if (I.dd) return factorize_dd_instance(I, coef_x, as_stream(hip_stream));
    return factorize_instance(p, I, coef_x, coef_y, as_stream(hip_stream));
  });
}

pr_status pr_fine_propagate(pr_problem p, const double* U_in, double* F_out, void* hip_stream) {
  return guarded([&]() -> pr_status {
    if (!p || !U_in || !F_out) return fail(PR_EINVAL, "NULL argument");
    if (U_in == F_out) return fail(PR_EINVAL, "U_in and F_out must not overlap");
    return fine_all(p, U_in, false, F_out, as_stream(hip_stream));
  });
}

pr_status pr_coarse_sweep(pr_problem p, const double* F, double* G_old, double* U, double* inc_dev,
                          void* hip_stream) {
  return guarded([&]() -> pr_status {
    if (!p || !G_old || !U) return fail(PR_EINVAL, "NULL argument");
    hipStream_t s = as_stream(hip_stream);
    return coarse_sweep_impl(p, F, G_old, U, reinterpret_cast<unsigned long long*>(inc_dev), s,
                             nullptr);
  });
}

pr_status pr_parareal_iterate(pr_problem p, const double* u0, double* U, int k_max, double tol,
                              int* k_done, double* inc, void* hip_stream) {
  return guarded([&]() -> pr_status {
    if (!p || !u0 || !U || !k_done || !inc) return fail(PR_EINVAL, "NULL argument");
    if (k_max < 0) return fail(PR_EINVAL, "k_max must be >= 0");
    if (!(tol >= 0)) return fail(PR_EINVAL, "tol must be >= 0");
    // the work runs on the library's stream once the caller's stream has drained
    HIPOK(hipStreamSynchronize(as_stream(hip_stream)));
    hipStream_t s = p->gstream;
    const int n = (int)p->inst.size();
    pr_status st = set_all_active(p, s);
    if (st != PR_OK) return st;
    for (int i = 0; i < n; i++) {
      Instance& I = *p->inst[i];
      HIPOK(launch_copy(u0 + I.off_u0, U + I.off_states, I.npts, s));
      k_done[i] = 0;
      inc[i] = 0.0;
    }
    st = coarse_sweep_impl(p, nullptr, p->Gold.p, U, p->d_inc, s, nullptr);  // initial guess
    if (st != PR_OK) return st;
    std::vector<char> active(n, 1);
    int n_active = n;
    // one parareal correction: F on all active slices, coarse sweep with the
    // correction and increment, device mask update, increment to the host
    auto correction = [&]() -> pr_status {
      pr_status r = fine_all(p, U, true, p->F.p, s, &active);
      if (r != PR_OK) return r;
      r = coarse_sweep_impl(p, p->F.p, p->Gold.p, U, p->d_inc, s, &active);
      if (r != PR_OK) return r;
      HIPOK(launch_mask_update(reinterpret_cast<const double*>(p->d_inc), p->d_active, n, tol, s));
      HIPOK(hipMemcpyAsync(p->h_inc, p->d_inc, n * sizeof(double), hipMemcpyDeviceToHost, s));
      return PR_OK;
    };
    // The captured correction bakes in which domain-decomposition instances are
    // still active (their kernels are skipped on the host); it is captured again
    // when that set changes, i.e. when such an instance converges.
    const bool graph = p->use_graph && !p->prof && k_max > 0;
    auto capture = [&]() -> pr_status {
      if (p->gexec) {
        (void)hipGraphExecDestroy(p->gexec);
        p->gexec = nullptr;
      }
      if (p->graph) {
        (void)hipGraphDestroy(p->graph);
        p->graph = nullptr;
      }
      HIPOK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      pr_status r = correction();
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(s, &g);
      if (r != PR_OK) {
        if (g) (void)hipGraphDestroy(g);
        return r;
      }
      HIPOK(e);
      p->graph = g;
      HIPOK(hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0));
      p->graph_tol = tol;
      p->graph_U = U;
      p->graph_active = active;
      return PR_OK;
    };
    auto dd_mask_changed = [&]() {
      if (!p->any_dd) return false;
      for (int i = 0; i < n; i++)
        if (p->inst[i]->dd && active[i] != p->graph_active[i]) return true;
      return false;
    };
    if (graph && (!p->gexec || p->graph_tol != tol || p->graph_U != U ||
                  p->graph_active.size() != active.size() || dd_mask_changed())) {
      st = capture();
      if (st != PR_OK) return st;
    }
    pr_status result = PR_OK;
    for (int k = 0; k < k_max && n_active > 0; k++) {
      if (graph) {
        if (dd_mask_changed()) {
          st = capture();
          if (st != PR_OK) return st;
        }
        HIPOK(hipGraphLaunch(p->gexec, s));
      } else {
        st = correction();
        if (st != PR_OK) return st;
      }
      HIPOK(hipStreamSynchronize(s));
      for (int i = 0; i < n; i++) {
        if (!active[i]) continue;
        const double v = p->h_inc[i];
        k_done[i] = k + 1;
        inc[i] = v;
        if (!std::isfinite(v)) result = fail(PR_ENUMERIC, "instance %d: non-finite increment", i);
        if (v < tol) {
          active[i] = 0;
          n_active--;
        }
      }
      if (result != PR_OK) break;
    }
    st = set_all_active(p, s);
    if (st != PR_OK) return st;
    return result;
  });
}

pr_status pr_set_option(pr_problem p, int option, int value) {
  return guarded([&]() -> pr_status {
    if (!p) return fail(PR_EINVAL, "NULL handle");
    switch (option) {
      case PR_OPT_GRAPH:
        if (value != 0 && value != 1) return fail(PR_EINVAL, "graph option must be 0 or 1");
        p->use_graph = value == 1;
        return PR_OK;
      case PR_OPT_FINE_CHUNK:
        if (value != 16 && value != 20 && value != 24 && value != 32)
          return fail(PR_EINVAL, "fine chunk must be 16, 20, 24 or 32");
        return apply_layout(p, p->lanes_cap, value, p->twisted);
      case PR_OPT_TWISTED:
        if (value != 0 && value != 1) return fail(PR_EINVAL, "twisted option must be 0 or 1");
        return apply_layout(p, p->lanes_cap, p->M, value == 1);
      case PR_OPT_GROUPED:
        if (value != 0 && value != 1) return fail(PR_EINVAL, "grouped option must be 0 or 1");
        p->grouped = value == 1;
        return apply_layout(p, p->lanes_cap, p->M, p->twisted);
      case PR_OPT_LANES:
        if (value != 0 && value != 8 && value != 16 && value != 32 && value != 64)
          return fail(PR_EINVAL, "lanes must be 0, 8, 16, 32 or 64");
        return apply_layout(p, value, p->M, p->twisted);
      case PR_OPT_PARTITIONED:
        if (value < 0 || value > 2) return fail(PR_EINVAL, "partitioned option must be 0, 1 or 2");
        p->part_sweeps = value;
        return apply_layout(p, p->lanes_cap, p->M, p->twisted);
      case PR_OPT_PARTITIONED_USED:
        return fail(PR_EINVAL, "option %d is read only", option);
      case PR_OPT_BLOCKS_PER_PASS:
        if (value < 0) return fail(PR_EINVAL, "blocks per pass must be >= 0");
        p->blocks_per_pass = value;
        return apply_layout(p, p->lanes_cap, p->M, p->twisted);
      default:
        return fail(PR_EINVAL, "unknown option %d", option);
    }
  });
}

pr_status pr_get_option(pr_problem p, int option, int* value) {
  return guarded([&]() -> pr_status {
    if (!p || !value) return fail(PR_EINVAL, "NULL argument");
    switch (option) {
      case PR_OPT_GRAPH: *value = p->use_graph ? 1 : 0; return PR_OK;
      case PR_OPT_FINE_CHUNK: *value = p->M; return PR_OK;
      case PR_OPT_TWISTED: *value = p->twisted ? 1 : 0; return PR_OK;
      case PR_OPT_GROUPED: *value = p->grouped ? 1 : 0; return PR_OK;
      case PR_OPT_LANES: *value = p->lanes_cap; return PR_OK;
      case PR_OPT_BLOCKS_PER_PASS: *value = p->blocks_per_pass; return PR_OK;
      case PR_OPT_PARTITIONED: *value = p->part_sweeps; return PR_OK;
      case PR_OPT_PARTITIONED_USED: {
        int c = 0;
        for (auto& I : p->inst) c += I->part ? 1 : 0;
        *value = c;
        return PR_OK;
      }
      default: return fail(PR_EINVAL, "unknown option %d", option);
    }
  });
}

pr_status pr_autotune(pr_problem p, void* hip_stream, int* lanes, int* chunk, float* best_ms) {
  return guarded([&]() -> pr_status {
    if (!p) return fail(PR_EINVAL, "NULL handle");
    hipStream_t s = as_stream(hip_stream);
    int Lmax = 8;
    for (auto& I : p->inst)
      if (!I->dd) Lmax = std::max(Lmax, I->Ldef);
    hipEvent_t e0, e1;
    HIPOK(hipEventCreate(&e0));
    HIPOK(hipEventCreate(&e1));
    float best = -1.f;
    int bl = p->lanes_cap, bm = p->M;
    bool btw = p->twisted;
    const bool prof = p->prof;
    p->prof = false;
    pr_status st = PR_OK;
    for (int L = 8; L <= Lmax && st == PR_OK; L <<= 1)
      for (int tw = 0; tw < 2 && st == PR_OK; tw++)
      for (int M : {16, 20, 24, 32}) {
        st = apply_layout(p, L == Lmax ? 0 : L, M, tw == 1);
        if (st != PR_OK) break;
        float ms_min = -1.f;
        for (int rep = 0; rep < 3 && st == PR_OK; rep++) {
          if (hipEventRecord(e0, s) != hipSuccess) { st = fail(PR_EDEVICE, "event record"); break; }
          st = fine_all(p, p->Gold.p, false, p->F.p, s);
          if (st != PR_OK) break;
          if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            st = fail(PR_EDEVICE, "event sync");
            break;
          }
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (rep > 0 && (ms_min < 0 || ms < ms_min)) ms_min = ms;  // first run warms up
        }
        if (st == PR_OK && (best < 0 || ms_min < best)) {
          best = ms_min;
          bl = L == Lmax ? 0 : L;
          bm = M;
          btw = tw == 1;
        }
      }
    p->prof = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PR_OK) return st;
    st = apply_layout(p, bl, bm, btw);
    if (st != PR_OK) return st;
    if (lanes) *lanes = bl;
    if (chunk) *chunk = bm;
    if (best_ms) *best_ms = best;
    return PR_OK;
  });
}

pr_status pr_sequential_fine(pr_problem p, const double* u0, double* U, void* hip_stream) {
  return guarded([&]() -> pr_status {
    if (!p || !u0 || !U) return fail(PR_EINVAL, "NULL argument");
    hipStream_t s = as_stream(hip_stream);
    const int n = (int)p->inst.size();
    for (int i = 0; i < n; i++) {
      Instance& I = *p->inst[i];
      const DimInst* dI = p->d_inst + i;
      HIPOK(launch_copy(u0 + I.off_u0, U + I.off_states, I.npts, s));
      if (I.dd) {
        for (int k = 0; k < I.d.n_slices; k++) {
          HIPOK(launch_copy(U + I.off_states + (size_t)k * I.npts, I.tmp.p, I.npts, s));
          for (int t = 0; t < I.d.fine_steps; t++) {
            if (I.dd2) {
              pr_status st = dd2_step_single(p, i, false, (long)k * I.d.fine_steps + t, s);
              if (st != PR_OK) return st;
              continue;
            }
            if (I.h.nforce)
              HIPOK(launch_force_state(dI, I.h, I.tmp.p, I.fgf.p, (long)k * I.d.fine_steps + t,
                                       (long)I.d.n_slices * I.d.fine_steps, s));
            pr_status st = dd_fie_step(p, I, false, 1, 0, s);
            if (st != PR_OK) return st;
          }
          HIPOK(launch_copy(I.tmp.p, U + I.off_states + (size_t)(k + 1) * I.npts, I.npts, s));
        }
        continue;
      }
      pr_status st = seq_fine_dim(p, i, u0 + I.off_u0, U + I.off_states, s);
      if (st != PR_OK) return st;
    }
    return PR_OK;
  });
}

pr_status pr_adjoint(pr_problem p, const double* u0, const double* lambda_T, double* grad_u0,
                     double* grad_coef, double* U_ckpt, void* hip_stream) {
  return guarded([&]() -> pr_status {
    pr_status st = check_adjoint_args(p, u0, lambda_T, grad_u0, grad_coef, "pr_adjoint");
    if (st != PR_OK) return st;
    Instance& I = *p->inst[0];
    const int nx = I.d.nx, ny = I.d.ny, N = I.d.n_slices, S = I.d.fine_steps;
    const size_t npts = I.npts;
    // workspace: post-x and post-y states of one slice's fine steps, checkpoints, lambda, mu
    if (I.adjWV.n != 2 * (size_t)S * npts) HIPOK(I.adjWV.alloc(2 * (size_t)S * npts));
    if (!U_ckpt && I.adjCkpt.n != (size_t)(N + 1) * npts) HIPOK(I.adjCkpt.alloc((size_t)(N + 1) * npts));
    if (I.adjLam.n != npts) HIPOK(I.adjLam.alloc(npts));
    if (I.adjMu.n != npts) HIPOK(I.adjMu.alloc(npts));
    if (I.adjGax.n != (size_t)ny * (nx + 1)) HIPOK(I.adjGax.alloc((size_t)ny * (nx + 1)));
    if (I.adjGay.n != (size_t)(ny + 1) * nx) HIPOK(I.adjGay.alloc((size_t)(ny + 1) * nx));
    AdjWork w{I.adjWV.p, I.adjWV.p + (size_t)S * npts, I.adjLam.p, I.adjMu.p, I.adjGax.p,
              I.adjGay.p, U_ckpt ? U_ckpt : I.adjCkpt.p};
    return adjoint_serial(p, u0, lambda_T, grad_u0, grad_coef, w, as_stream(hip_stream));
  });
}

pr_status pr_adjoint_noalloc(pr_problem p, const double* u0, const double* lambda_T,
                             double* grad_u0, double* grad_coef, double* U_ckpt,
                             void* hip_stream) {
  return guarded([&]() -> pr_status {
    pr_status st = check_adjoint_args(p, u0, lambda_T, grad_u0, grad_coef, "pr_adjoint_noalloc");
    if (st != PR_OK) return st;
    Instance& I = *p->inst[0];
    const int nx = I.d.nx, ny = I.d.ny, N = I.d.n_slices, S = I.d.fine_steps;
    const size_t npts = I.npts;
    // carve the workspace out of this GPU's scratch array, each part 256-byte aligned
    const size_t parts[7] = {(size_t)S * npts, (size_t)S * npts, npts, npts,
                             (size_t)ny * (nx + 1), (size_t)(ny + 1) * nx,
                             U_ckpt ? 0 : (size_t)(N + 1) * npts};
    size_t need = 0;
    for (size_t n : parts) need += (n + 31) / 32 * 32;
    if (need > kNoAllocScratchDoubles)
      return fail(PR_EINVAL,
                  "pr_adjoint_noalloc: this problem needs %zu doubles of scratch (2 s + 2 states, "
                  "the face gradients%s), above the library's fixed %zu",
                  need, U_ckpt ? "" : " and N + 1 checkpoints", (size_t)kNoAllocScratchDoubles);
    double* base = nullptr;
    st = device_scratch(&base);
    if (st != PR_OK) return st;
    double* q[7];
    for (int k = 0; k < 7; k++) {
      q[k] = base;
      base += (parts[k] + 31) / 32 * 32;
    }
    AdjWork w{q[0], q[1], q[2], q[3], q[4], q[5], U_ckpt ? U_ckpt : q[6]};
    return adjoint_serial(p, u0, lambda_T, grad_u0, grad_coef, w, as_stream(hip_stream));
  });
}

// Parallel-in-time adjoint (not in the paper; derived from the transpose of
// eq. FIE_method). One FIE step is V = By^{-1} Bx^{-1} (U + dt F) with
// symmetric Bx, By, so the adjoint of the fine map of one slice is s steps of
// "y solve, then x solve" — the forward map of the transposed grid. The
// boundary adjoints lambda_n = F_n^T lambda_{n+1} are therefore the states of
// the transposed problem started from lambda_T^T: its sequential fine solve
// (k_max = 0, exact) or parareal (k_max > 0, tolerance tol), run through an
// internal handle. With lambda_{n+1} known for every slice, all slices
// recompute their forward steps at once (batched sweeps, every step's state
// kept) and run their reverse steps at once, accumulating the face gradients
// over slices.
pr_status pr_adjoint_parallel(pr_problem p, const double* u0, const double* lambda_T,
                              double* grad_u0, double* grad_coef, double* U_ckpt, int k_max,
                              double tol, int* k_done, void* hip_stream) {
  return guarded([&]() -> pr_status {
    if (!p || !u0 || !lambda_T || !grad_u0 || !grad_coef) return fail(PR_EINVAL, "NULL argument");
    if (p->inst.size() != 1)
      return fail(PR_EUNSUPPORTED, "pr_adjoint_parallel needs a single-instance handle");
    if (k_max < 0 || !(tol >= 0)) return fail(PR_EINVAL, "k_max must be >= 0 and tol >= 0");
    Instance& I = *p->inst[0];
    if (I.dd || I.d.dim != 2)
      return fail(PR_EUNSUPPORTED, "pr_adjoint_parallel supports 2D dimensional splitting");
    if (I.d.fine != PR_FIE)
      return fail(PR_EUNSUPPORTED, "pr_adjoint_parallel supports the FIE fine propagator only");
    hipStream_t s = as_stream(hip_stream);
    const int nx = I.d.nx, ny = I.d.ny, N = I.d.n_slices, S = I.d.fine_steps;
    const size_t npts = I.npts;
    const DimInst& h = I.h;
    const pr_problem_s::Group& g = p->groups.at(0);
    HIPOK(hipStreamSynchronize(s));
    // 1. workspaces and per-step descriptors (the library's work of earlier calls
    //    has drained: nothing reads them while they change)
    const size_t slabs = (size_t)h.B * h.slab;
    const size_t nsx = (size_t)h.B * ny * h.Px * h.L, nsy = (size_t)h.B * nx * h.Py * h.L;
    if (I.pSnap.n != 2 * (size_t)S * slabs || I.pSigX.n != (size_t)S * nsx) {
      HIPOK(I.pSnap.alloc(2 * (size_t)S * slabs));
      HIPOK(I.pSigX.alloc((size_t)S * nsx));
      HIPOK(I.pSigY.alloc((size_t)S * nsy));
      HIPOK(I.pInit.alloc(slabs));
      HIPOK(I.pLam.alloc(slabs));
      HIPOK(I.pSigXa.alloc(nsx));
      HIPOK(I.pSigYa.alloc(nsy));
    }
    auto snap = [&](int k) { return I.pSnap.p + (size_t)k * slabs; };
    // descriptors: [0] checkpoints, [1 + 2t] x step t, [2 + 2t] y step t,
    // [2S + 1 + 2t] W_t, [2S + 2 + 2t] V_t, [4S + 1] adjoint workspace
    std::vector<DimInst>& D = I.pDescHost;
    D.assign(4 * (size_t)S + 2, h);
    for (auto& d : D) {
      d.active = nullptr;
      d.zout = 0;
    }
    D[0].Z = I.pInit.p;
    for (int t = 0; t < S; t++) {
      DimInst& dx = D[1 + 2 * t];
      dx.Z = t == 0 ? I.pInit.p : snap(2 * t - 1);
      dx.zout = (long)(snap(2 * t) - dx.Z);
      dx.sigY = t == 0 ? I.pSigY.p : I.pSigY.p + (size_t)(t - 1) * nsy;
      dx.sigX = I.pSigX.p + (size_t)t * nsx;
      DimInst& dy = D[2 + 2 * t];
      dy.Z = snap(2 * t);
      dy.zout = (long)(snap(2 * t + 1) - dy.Z);
      dy.sigX = I.pSigX.p + (size_t)t * nsx;
      dy.sigY = I.pSigY.p + (size_t)t * nsy;
      DimInst& gw = D[2 * S + 1 + 2 * t];
      gw.Z = snap(2 * t);
      gw.sigX = I.pSigX.p + (size_t)t * nsx;
      DimInst& gv = D[2 * S + 2 + 2 * t];
      gv.Z = snap(2 * t + 1);
      gv.sigY = I.pSigY.p + (size_t)t * nsy;
    }
    DimInst& da = D[4 * S + 1];
    da.Z = I.pLam.p;
    da.sigX = I.pSigXa.p;
    da.sigY = I.pSigYa.p;
    da.nforce = 0;
    HIPOK(I.pDesc.upload(D));
    // 2. transposed problem (once per handle): nx <-> ny, coefficients transposed
    if (!p->adjT) {
      pr_problem_desc dT = I.d;
      dT.nx = ny;
      dT.ny = nx;
      dT.n_forcing = 0;
      dT.forcing_space = dT.forcing_time_fine = dT.forcing_time_coarse = nullptr;
      dT.rho = nullptr;
      if (I.d.coef_mode == PR_COEF_NODAL_LOG) {
        HIPOK(I.pCoefT0.alloc((size_t)(nx + 2) * (ny + 2)));
        HIPOK(launch_transpose_states(I.theta.p, I.pCoefT0.p, nx + 2, ny + 2, 1, s));
        dT.coef_x = I.pCoefT0.p;
        dT.coef_y = nullptr;
      } else {  // x-faces of the transposed grid are the y-faces, and back
        HIPOK(I.pCoefT0.alloc((size_t)nx * (ny + 1)));
        HIPOK(I.pCoefT1.alloc((size_t)(nx + 1) * ny));
        HIPOK(launch_transpose_states(I.ay.p, I.pCoefT0.p, nx, ny + 1, 1, s));
        HIPOK(launch_transpose_states(I.ax.p, I.pCoefT1.p, nx + 1, ny, 1, s));
        dT.coef_x = I.pCoefT0.p;
        dT.coef_y = I.pCoefT1.p;
      }
      HIPOK(hipStreamSynchronize(s));
      pr_problem hT = nullptr;
      pr_status st = pr_create_problem(&dT, 1, hip_stream, &hT);
      if (st != PR_OK) return st;
      p->adjT = hT;
    }
    // 3. boundary adjoints: states of the transposed problem from lambda_T^T.
    //    The exact chain runs on a second stream, beside the forward checkpoints
    //    of step 4 (the two serial chains are independent).
    if (!p->astream) {
      HIPOK(hipStreamCreateWithFlags(&p->astream, hipStreamNonBlocking));
      HIPOK(hipEventCreateWithFlags(&p->aev[0], hipEventDisableTiming));
      HIPOK(hipEventCreateWithFlags(&p->aev[1], hipEventDisableTiming));
    }
    if (I.pBnd.n != (size_t)(N + 1) * npts) {
      HIPOK(I.pBnd.alloc((size_t)(N + 1) * npts));
      HIPOK(I.pBndT.alloc((size_t)(N + 1) * npts));
      HIPOK(I.pLamIn.alloc((size_t)N * npts));
    }
    HIPOK(launch_transpose_states(lambda_T, I.pBndT.p, nx, ny, 1, s));  // u0 of the transposed problem
    pr_status st = PR_OK;
    int kd = 0;
    hipStream_t bs = s;  // stream of the boundary-adjoint chain
    if (k_max == 0) {
      bs = p->astream;
      HIPOK(hipEventRecord(p->aev[0], s));
      HIPOK(hipStreamWaitEvent(bs, p->aev[0], 0));
      st = pr_sequential_fine(p->adjT, I.pBndT.p, I.pBndT.p, bs);
    } else {
      double incT = 0.0;
      HIPOK(launch_copy(I.pBndT.p, I.pBnd.p, npts, s));  // pr_parareal_iterate reads u0 separately
      st = pr_parareal_iterate(p->adjT, I.pBnd.p, I.pBndT.p, k_max, tol, &kd, &incT, hip_stream);
    }
    if (st != PR_OK) return st;
    if (k_done) *k_done = kd;
    // transposed state m is lambda_{N-m}^T
    HIPOK(launch_transpose_states(I.pBndT.p, I.pBnd.p, ny, nx, N + 1, bs));
    for (int n = 0; n < N; n++)  // slice n ends with lambda_{n+1} = state N-1-n
      HIPOK(launch_copy(I.pBnd.p + (size_t)(N - 1 - n) * npts, I.pLamIn.p + (size_t)n * npts, npts,
                        bs));
    if (bs != s) HIPOK(hipEventRecord(p->aev[1], bs));
    // 4. forward checkpoints at the slice boundaries (exact sequential fine solve)
    if (!U_ckpt && I.adjCkpt.n != (size_t)(N + 1) * npts) HIPOK(I.adjCkpt.alloc((size_t)(N + 1) * npts));
    double* ckpt = U_ckpt ? U_ckpt : I.adjCkpt.p;
    st = seq_fine_dim(p, 0, u0, ckpt, s);
    if (st != PR_OK) return st;
    if (bs != s) HIPOK(hipStreamWaitEvent(s, p->aev[1], 0));
    const DimInst* Dd = I.pDesc.p;
    // 5. recompute every forward step of every slice (sources included)
    HIPOK(launch_to_interleaved(Dd, h, ckpt, s));
    for (int t = 0; t < S; t++) {
      PhaseTimer pt(p, PH_FINE, s);
      HIPOK(launch_fine_sweep(Dd + 1 + 2 * t, g.d_work[0], g.n_work[0], g.L, g.M, 0, t > 0, t, s, 0,
                              g.ft != 0, p->twisted, g.grouped, g.long_lines));
      HIPOK(launch_fine_sweep(Dd + 2 + 2 * t, g.d_work[1], g.n_work[1], g.L, g.M, 1, 1, t, s, 0,
                              false, p->twisted, g.grouped, g.long_lines));
    }
    // 6. reverse steps of every slice from lambda_{n+1}: y solve, face gradients
    //    with V_t, x solve, face gradients with W_t
    if (I.adjGax.n != (size_t)ny * (nx + 1)) HIPOK(I.adjGax.alloc((size_t)ny * (nx + 1)));
    if (I.adjGay.n != (size_t)(ny + 1) * nx) HIPOK(I.adjGay.alloc((size_t)(ny + 1) * nx));
    HIPOK(launch_fill_zero(I.adjGax.p, I.adjGax.n, s));
    HIPOK(launch_fill_zero(I.adjGay.p, I.adjGay.n, s));
    const double hx = 1.0 / (nx + 1), hy = 1.0 / (ny + 1);
    const double cx = I.dt / (hx * hx), cy = I.dt / (hy * hy);
    const DimInst* Da = Dd + 4 * S + 1;
    HIPOK(launch_to_interleaved(Da, h, I.pLamIn.p, s));
    for (int t = S - 1; t >= 0; t--) {
      {
        PhaseTimer pt(p, PH_FINE, s);
        HIPOK(launch_fine_sweep(Da, g.d_work[1], g.n_work[1], g.L, g.M, 1, t < S - 1, t, s, 0, false,
                                p->twisted, g.grouped, g.long_lines));
      }
      HIPOK(launch_grad_faces(1, Da, Dd + 2 * S + 2 + 2 * t, h, cy, I.adjGay.p, s));
      {
        PhaseTimer pt(p, PH_FINE, s);
        HIPOK(launch_fine_sweep(Da, g.d_work[0], g.n_work[0], g.L, g.M, 0, 1, t, s, 0, false,
                                p->twisted, g.grouped, g.long_lines));
      }
      HIPOK(launch_grad_faces(0, Da, Dd + 2 * S + 1 + 2 * t, h, cx, I.adjGax.p, s));
    }
    HIPOK(launch_slice_xcorr(Da, h, 0, grad_u0, s));  // lambda_0
    if (I.d.coef_mode == PR_COEF_NODAL_LOG) {
      HIPOK(launch_theta_chain(I.theta.p, I.adjGax.p, I.adjGay.p, nx, ny, grad_coef, s));
    } else {
      HIPOK(launch_copy(I.adjGax.p, grad_coef, I.adjGax.n, s));
      HIPOK(launch_copy(I.adjGay.p, grad_coef + I.adjGax.n, I.adjGay.n, s));
    }
    return PR_OK;
  });
}

}  // extern "C"
