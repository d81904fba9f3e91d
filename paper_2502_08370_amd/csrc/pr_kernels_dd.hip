// HIP kernels (gfx950, wave64, FP64) for the domain-decomposition splitting
// in 1D (arXiv 2502.08370, section 2.1: sub-operators L_k u = (rho_k a u_x)_x
// with a partition of unity rho_k; eq. FIE_method for the substeps).
//
// A colour's substep is one tridiagonal system per connected component of the
// colour, identity elsewhere (section 2.2, last paragraphs). Components are
// long (2^17+ nodes) and few, so each is cut into segments of kDDSeg nodes and
// solved in three phases (segment solves, carry scans, carry corrections; see
// pr_internal.h). Data are slice-interleaved Z[b][node][l] so that a wave whose
// lanes are (segment, slice) moves contiguous 8*L-byte runs.
#include "pr_internal.h"

namespace prk {

namespace {

constexpr int kWave = 64;

#define GLOBAL __attribute__((address_space(1)))
typedef GLOBAL double gdouble;
__device__ __forceinline__ gdouble* gp(double* p) { return (gdouble*)p; }
__device__ __forceinline__ const gdouble* gp(const double* p) { return (const gdouble*)p; }

__device__ __forceinline__ double lane_value(double v, int src) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ void affine_scan_up(double& a, double& b, int lane) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    double ap = __shfl_up(a, off, kWave);
    double bp = __shfl_up(b, off, kWave);
    if (lane >= off) {
      b = fma(a, bp, b);
      a = a * ap;
    }
  }
}

__device__ __forceinline__ void affine_scan_down(double& a, double& b, int lane) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    double an = __shfl_down(a, off, kWave);
    double bn = __shfl_down(b, off, kWave);
    if (lane + off < kWave) {
      b = fma(a, bn, b);
      a = a * an;
    }
  }
}

// The same scans within groups of WIDTH lanes (lane = index in the group).
template <int WIDTH>
__device__ __forceinline__ void group_scan_up(double& a, double& b, int lane) {
#pragma unroll
  for (int off = 1; off < WIDTH; off <<= 1) {
    double ap = __shfl_up(a, off, WIDTH);
    double bp = __shfl_up(b, off, WIDTH);
    if (lane >= off) {
      b = fma(a, bp, b);
      a = a * ap;
    }
  }
}

template <int WIDTH>
__device__ __forceinline__ void group_scan_down(double& a, double& b, int lane) {
#pragma unroll
  for (int off = 1; off < WIDTH; off <<= 1) {
    double an = __shfl_down(a, off, WIDTH);
    double bn = __shfl_down(b, off, WIDTH);
    if (lane + off < WIDTH) {
      b = fma(a, bn, b);
      a = a * an;
    }
  }
}

// Single-state segment kernels: a segment per group of kDDSeg lanes, lane = node.
constexpr int kSegsPerWave = kWave / kDDSeg;
static_assert(kWave % kDDSeg == 0, "segments tile a wave");

__device__ __forceinline__ unsigned long long abs_bits(double v) {
  return static_cast<unsigned long long>(__double_as_longlong(fabs(v)));
}

// ----------------------------------------------------------------- set-up ---

// w[k][f] = rho_k(face f) * a(face f)
__global__ void k_dd_faces(const double* __restrict__ rho, const double* __restrict__ a, int n,
                           int n_colors, double* __restrict__ w) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  long per = n + 1;
  if (t < per * n_colors) w[t] = rho[t] * a[t % per];
}

// LU of I - tau A_k restricted to one component (nodes lo..hi), one thread
// per component. Faces just outside a component carry rho_k = 0, so the
// restricted matrix is the exact block of the substep. The matrix is
// symmetric, so the forward multiplier e_i = w_i / u_{i-1} equals
// g_{i-1} = w_i r_{i-1}; it is formed as that product, and the kernels read it
// as G[i-1] (0 at a component's first node, where the previous entry is the
// end of another component or untouched zero).
__global__ void k_dd_factorize(const double* __restrict__ w, int n,
                               const int* __restrict__ comp_lo, const int* __restrict__ comp_hi,
                               const int* __restrict__ comp_colour, int n_comps,
                               double tau_over_h2, double* __restrict__ R,
                               double* __restrict__ G) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_comps) return;
  const int lo = comp_lo[c], hi = comp_hi[c], k = comp_colour[c];
  const double* wk = w + (long)k * (n + 1);
  const long base = (long)k * n;
  double r_prev = 0.0;
  double wl = tau_over_h2 * wk[lo];
  for (int i = lo; i <= hi; i++) {
    double wr = tau_over_h2 * wk[i + 1];
    double diag = 1.0 + wl + wr;
    double e = (i == lo) ? 0.0 : wl * r_prev;
    double u = diag - wl * e;
    double r = 1.0 / u;
    R[base + i] = r;
    G[base + i] = (i < hi) ? wr * r : 0.0;
    r_prev = r;
    wl = wr;
  }
}

// Per segment: psi (product of e over the segment), chi_i = r_i psi_i +
// g_i chi_{i+1} (chi past the end 0) and phi_i = g_i phi_{i+1} (phi past the
// end 1), with psi_i the product of e from the segment start to i.
__global__ void k_dd_segfactors(const DDSeg* __restrict__ segs, const int* __restrict__ seg_colour,
                                int n_segs, int n, const double* __restrict__ R,
                                const double* __restrict__ G,
                                double* __restrict__ CHI, double* __restrict__ PHI,
                                double* __restrict__ PSIE, double* __restrict__ CHIA,
                                double* __restrict__ PHIA) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_segs) return;
  const DDSeg sg = segs[s];
  const long base = (long)seg_colour[s] * n + sg.lo;
  double p = 1.0;
  for (int t = 0; t < sg.len; t++) {  // psi kept in CHI until the backward pass
    p = p * (sg.lo + t > 0 ? G[base + t - 1] : 0.0);  // e = g of the previous node
    CHI[base + t] = p;
  }
  PSIE[s] = p;
  double chi = 0.0, phi = 1.0;
  for (int t = sg.len - 1; t >= 0; t--) {
    chi = fma(G[base + t], chi, R[base + t] * CHI[base + t]);
    phi = G[base + t] * phi;
    CHI[base + t] = chi;
    PHI[base + t] = phi;
  }
  CHIA[s] = chi;
  PHIA[s] = phi;
}

// ------------------------------------------------------------- phase 1 ---
// Slice-interleaved workspace, one workgroup per (run, slice block) with
// kDDRun * L lanes. Every wave solves G segments of the run with zero carries:
// forward elimination (tilde y) and back substitution (tilde z) in place. The
// loaded values first receive the pending correction chi Yin + phi Xin of the
// segment's source (see DDInst), and the segment's own correction is left
// pending in turn. Then one lane per slice chains the run's segments (tilde y
// at each segment's last node and tilde z at its first node are staged in
// LDS): Y before segment t = A_t RY + B_t (A_t = SA_t, the product of PSIE
// before t), X after segment t = C_t RX + D_t RY + E_t with
//   X after t-1 = PHIA_t (X after t) + CHIA_t (Y before t) + tilde z_first,t,
// which leaves B_t, E_t in Yp, Xp and the run's maps (Y after the run =
// RP RY + RQ, X at its first node = RU RX + RV RY + RW) for the scan over the
// component's runs. C_t and D_t are the slice-independent SC_t, SD_t.
template <int L>
__global__ __launch_bounds__(kDDRun* L) void k_dd_local_run(const DDInst* __restrict__ insts,
                                                            DDFactors f, int colour,
                                                            int run_begin, int stale_ok) {
  constexpr int G = kWave / L;  // segments per wave
  constexpr int M = kDDSeg;
  constexpr int NW = kDDRun / G;  // waves per workgroup
  constexpr int NQ = (G * M + kWave - 1) / kWave;
  static_assert(kDDRun % G == 0, "a run is a whole number of waves");
  __shared__ double sE[NW][G][M + 1], sR[NW][G][M + 1], sG[NW][G][M + 1];
  __shared__ double sC[NW][G][M + 1], sP[NW][G][M + 1];
  __shared__ double sYb[kDDRun][L], sZa[kDDRun][L];
  __shared__ double sF[4][kDDRun];  // the run's PSIE, CHIA, PHIA, SA
  const DDInst& I = insts[0];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int gsub = lane / L, sl = lane - gsub * L;
  const int b = blockIdx.y;
  const int ri = run_begin + blockIdx.x;
  const DDRunRec* rec = I.run_recs + ri;
  const int rlen = rec->len, seg0 = rec->seg0;  // workgroup-uniform
  const int t0 = wv * G;        // the wave's first segment in the run
  const int tr = t0 + gsub;     // the lane's segment in the run
  const bool active = tr < rlen;
  // the lane's segment, its source and the source's run, from the run record
  const int slo = rec->lo[tr], scnt = rec->cnt[tr];
  const int src = rec->src[stale_ok][tr], sr = rec->srun[stale_ok][tr];
  const long cb = (long)colour * I.n;
  // the lane's segment values (the longest-latency loads)
  gdouble* zb = gp(I.Z) + b * I.slab + (long)slo * L + sl;
  double v[M];
#pragma unroll
  for (int t = 0; t < M; t++) {
    const double x = zb[(long)(t < scnt ? t : 0) * L];
    v[t] = t < scnt ? x : 0.0;
  }
  // carries of the source segment, from its run's carries and its slice parts
  // (read before this workgroup overwrites the slice parts of its own run: a
  // segment's source in its own colour is the segment itself)
  const int sc = src >= 0 ? src : 0;
  const long si = ((long)b * I.n_segs + sc) * L + sl;
  const long sri = ((long)b * I.n_runs + sr) * L + sl;
  const double yp = gp(I.Yp)[si], xp = gp(I.Xp)[si];
  const double ry = gp(I.RY)[sri], rx = gp(I.RX)[sri];
  const double fa = gp(f.SA)[sc], fc = gp(f.SC)[sc], fd = gp(f.SD)[sc];
  if (threadIdx.x < 4 * kDDRun) {  // the run's factors for the chaining below
    const int k = threadIdx.x / kDDRun, t = threadIdx.x - k * kDDRun;
    const int s = seg0 + (t < rlen ? t : 0);
    const gdouble* src_f = gp(k == 0 ? f.PSIE : (k == 1 ? f.CHIA : (k == 2 ? f.PHIA : f.SA)));
    sF[k][t] = src_f[s];
  }
  // factors of the wave's segments; padded positions act as identity and
  // carry no pending correction
  const gdouble* R = gp(f.R) + cb;
  const gdouble* Gf = gp(f.G) + cb;
  const gdouble* PC = gp(stale_ok ? f.PC1 : f.PC0) + cb;
  const gdouble* PP = gp(stale_ok ? f.PP1 : f.PP0) + cb;
#pragma unroll
  for (int qq = 0; qq < NQ; qq++) {
    const int q = lane + qq * kWave;
    if (q < G * M) {
      const int g = q / M, t = q - g * M;
      const int tg = t0 + g;
      const int glo = rec->lo[tg], gcnt = rec->cnt[tg];  // cnt = 0 past the run's end
      const bool ok = t < gcnt;
      const long node = glo + (ok ? t : 0);
      // e = g of the previous node (same cache lines as g)
      const double e = Gf[node > 0 ? node - 1 : 0], r = R[node], gg = Gf[node];
      const double c = PC[node], p = PP[node];
      sE[wv][g][t] = ok ? (node > 0 ? e : 0.0) : 1.0;
      sR[wv][g][t] = ok ? r : 0.0;
      sG[wv][g][t] = ok ? gg : 0.0;
      sC[wv][g][t] = ok ? c : 0.0;
      sP[wv][g][t] = ok ? p : 0.0;
    }
  }
  const double ys = src >= 0 ? fma(fa, ry, yp) : 0.0;
  const double xs = src >= 0 ? fma(fc, rx, fma(fd, ry, xp)) : 0.0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the wave's factor staging
#pragma unroll
  for (int t = 0; t < M; t++) v[t] = fma(sP[wv][gsub][t], xs, fma(sC[wv][gsub][t], ys, v[t]));
  double y = 0.0;
#pragma unroll
  for (int t = 0; t < M; t++) {
    y = fma(sE[wv][gsub][t], y, v[t]);
    v[t] = y;
  }
  double z = 0.0;
#pragma unroll
  for (int t = M - 1; t >= 0; t--) {
    z = fma(sG[wv][gsub][t], z, sR[wv][gsub][t] * v[t]);
    v[t] = z;
  }
  if (active) {  // streaming stores: each value is read once, by a later substep
#pragma unroll
    for (int t = 0; t < M; t++)
      if (t < scnt) __builtin_nontemporal_store(v[t], &zb[(long)t * L]);
  }
  sYb[tr][sl] = y;
  sZa[tr][sl] = v[0];
  __syncthreads();
  if (threadIdx.x < L) {  // one lane per slice; the run's factors are uniform
    const int l = threadIdx.x;
    double A = 1.0, Bq = 0.0;
    const long base = (long)b * I.n_segs * L + l;
    for (int t = 0; t < rlen; t++) {  // B_t replaces tilde y in LDS
      const double yb = sYb[t][l];
      sYb[t][l] = Bq;
      gp(I.Yp)[base + (long)(seg0 + t) * L] = Bq;
      Bq = fma(sF[0][t], Bq, yb);
      A = sF[0][t] * A;
    }
    double C = 1.0, D = 0.0, E = 0.0;
    for (int t = rlen - 1; t >= 0; t--) {
      const double pa = sF[2][t], ca = sF[1][t];
      gp(I.Xp)[base + (long)(seg0 + t) * L] = E;
      E = fma(pa, E, fma(ca, sYb[t][l], sZa[t][l]));
      D = fma(pa, D, ca * sF[3][t]);
      C = pa * C;
    }
    const long ridx = ((long)b * I.n_runs + ri) * L + l;
    gp(I.RP)[ridx] = A;
    gp(I.RQ)[ridx] = Bq;
    gp(I.RU)[ridx] = C;
    gp(I.RV)[ridx] = D;
    gp(I.RW)[ridx] = E;
  }
}

// Carries of every segment (and slice) after the last substep, from its run's
// carries and its slice parts, for the final transpose: one thread per entry.
__global__ void k_dd_final_carries(const DDInst* __restrict__ insts, DDFactors f) {
  const DDInst& I = insts[0];
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long per = (long)I.n_segs * I.L;
  if (t >= (long)I.B * per) return;
  const int b = (int)(t / per);
  const long r = t - b * per;
  const int s = (int)(r / I.L), l = (int)(r - (long)s * I.L);
  const long ri = ((long)b * I.n_runs + I.seg_run[s]) * I.L + l;
  const double ry = gp(I.RY)[ri], rx = gp(I.RX)[ri];
  gp(I.Yin)[t] = fma(gp(f.SA)[s], ry, gp(I.Yp)[t]);
  gp(I.Xin)[t] = fma(gp(f.SC)[s], rx, fma(gp(f.SD)[s], ry, gp(I.Xp)[t]));
}

// SA, SC, SD of every run's segments (one thread per run): the same products
// as k_dd_local_run forms, in the same order.
__global__ void k_dd_runfactors(const DDInst* __restrict__ insts, DDFactors f,
                                double* __restrict__ SA, double* __restrict__ SC,
                                double* __restrict__ SD) {
  const DDInst& I = insts[0];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= I.n_runs) return;
  const DDRun rn = I.runs[r];
  double A = 1.0;
  for (int t = 0; t < rn.len; t++) {
    SA[rn.seg0 + t] = A;
    A = f.PSIE[rn.seg0 + t] * A;
  }
  double C = 1.0, D = 0.0;
  for (int t = rn.len - 1; t >= 0; t--) {
    const int s = rn.seg0 + t;
    SC[s] = C;
    SD[s] = D;
    D = fma(f.PHIA[s], D, f.CHIA[s] * SA[s]);
    C = f.PHIA[s] * C;
  }
}

// Pending-correction factors: for each node of each segment, chi and phi of
// the colour whose correction the node carries when the segment's colour loads
// it (first step / later steps); for each node, those of its final correction.
__global__ void k_dd_pending(const DDInst* __restrict__ insts, DDFactors f,
                             double* __restrict__ PC0, double* __restrict__ PP0,
                             double* __restrict__ PC1, double* __restrict__ PP1,
                             double* __restrict__ FC, double* __restrict__ FP) {
  const DDInst& I = insts[0];
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nseg_nodes = (long)I.n_segs * kDDSeg;
  if (t < nseg_nodes) {
    const int si = (int)(t / kDDSeg), j = (int)(t - (long)si * kDDSeg);
    const DDSeg sg = I.segs[si];
    if (j >= sg.len) return;
    const long node = sg.lo + j, at = (long)sg.colour * I.n + node;
    const int s0 = I.seg_src0[si], s1 = I.seg_src1[si];
    PC0[at] = s0 >= 0 ? f.CHI[(long)I.segs[s0].colour * I.n + node] : 0.0;
    PP0[at] = s0 >= 0 ? f.PHI[(long)I.segs[s0].colour * I.n + node] : 0.0;
    PC1[at] = s1 >= 0 ? f.CHI[(long)I.segs[s1].colour * I.n + node] : 0.0;
    PP1[at] = s1 >= 0 ? f.PHI[(long)I.segs[s1].colour * I.n + node] : 0.0;
  } else if (t < nseg_nodes + I.n) {
    const long node = t - nseg_nodes;
    const int fs = I.fin_seg[node];
    FC[node] = fs >= 0 ? f.CHI[(long)I.segs[fs].colour * I.n + node] : 0.0;
    FP[node] = fs >= 0 ? f.PHI[(long)I.segs[fs].colour * I.n + node] : 0.0;
  }
}

// Final transpose of the deferred fine substeps: F[slice][node] = Z[b][node][l]
// + chi Yin + phi Xin of the node's last segment (the carries formed by
// k_dd_final_carries); one block of 4 waves per (64-node tile, slice block).
__global__ __launch_bounds__(4 * kWave) void k_dd_from_interleaved(
    const DDInst* __restrict__ insts, DDFactors f, double* __restrict__ F) {
  __shared__ double tile[64][65];
  const DDInst& I = insts[0];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int i0 = blockIdx.x * 64, b = blockIdx.y;
  const int L = I.L, lg = 31 - __clz(L);
  const int cnt = min(64, I.n - i0), n = cnt * L;
  const gdouble* Zb = gp(I.Z) + b * I.slab + (long)i0 * L;
  constexpr int kIt = 64 * 64 / (4 * kWave);
  double z[kIt], c[kIt], p[kIt], yi[kIt], xi[kIt];
#pragma unroll
  for (int u = 0; u < kIt; u++) {
    const int q = tid + 4 * kWave * u;
    const bool ok = q < n;
    const int t = ok ? q >> lg : 0, sl = q & (L - 1);
    const int node = i0 + t;
    const int fs0 = I.fin_seg[node];
    const int fs = fs0 >= 0 ? fs0 : 0;  // FC = FP = 0 when there is none
    const long bi = ((long)b * I.n_segs + fs) * L + sl;
    z[u] = Zb[ok ? q : 0];
    c[u] = gp(f.FC)[node];
    p[u] = gp(f.FP)[node];
    yi[u] = gp(I.Yin)[bi];
    xi[u] = gp(I.Xin)[bi];
  }
#pragma unroll
  for (int u = 0; u < kIt; u++) {
    const int q = tid + 4 * kWave * u;
    if (q < n) tile[q & (L - 1)][q >> lg] = fma(p[u], xi[u], fma(c[u], yi[u], z[u]));
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kIt; u++) {
    const int sl = w + 4 * u, slice = b * L + sl;
    if (sl < L && slice < I.N && lane < cnt)
      __builtin_nontemporal_store(tile[sl][lane], &F[(long)slice * I.n + i0 + lane]);
  }
}

// ------------------------------------------------------------- phase 2 ---
// Carry resolution per (component, slice): Y_s = Yb_s + psi_s Y_{s-1} over the
// component's segments, then X_s = Za_s + chi_s Y_{s-1} + phi_s X_{s+1}
// backwards, over runs of kDDRun segments (see pr_internal.h): each run's maps
// and the slice parts of its segments' carries (formed by the segment solves'
// workgroups, k_dd_local_run and k_dd_local_run1), then the scan over each
// component's runs (below); a segment's carries are formed where they are used.

// 2b: chains the runs of one component for one slice, 64 runs per wave step.
// Components of up to kScanChunks * 64 runs (2^17-node components in 32-node
// segments have 257) take a path that issues every load up front and keeps the
// forward results in registers.
constexpr int kScanChunks = 5;

__global__ __launch_bounds__(kWave) void k_dd_runscan(const DDInst* __restrict__ insts,
                                                      const int* __restrict__ comp_run_first,
                                                      const int* __restrict__ comp_run_count) {
  const DDInst& I = insts[0];
  const int lane = threadIdx.x;
  const int comp = blockIdx.x;
  const int slice = blockIdx.y;  // b * L + l
  const int b = slice / I.L, sl = slice - b * I.L;
  const int first = comp_run_first[comp], count = comp_run_count[comp];
  const long rb = (long)b * I.n_runs;
  const int nch = (count + kWave - 1) / kWave;
  if (nch <= kScanChunks) {
    double rp[kScanChunks], rq[kScanChunks], ru[kScanChunks], rv[kScanChunks], rw[kScanChunks];
    double ry[kScanChunks];
#pragma unroll
    for (int ch = 0; ch < kScanChunks; ch++) {
      const int r = first + ch * kWave + lane;
      const bool ok = r < first + count;
      const long ri = (rb + (ok ? r : first)) * I.L + sl;
      const double p = gp(I.RP)[ri], q = gp(I.RQ)[ri];
      const double u = gp(I.RU)[ri], v = gp(I.RV)[ri], w = gp(I.RW)[ri];
      rp[ch] = ok ? p : 1.0;  // identity past the end (forward)
      rq[ch] = ok ? q : 0.0;
      ru[ch] = ok ? u : 0.0;  // X = 0 after the component (backward)
      rv[ch] = ok ? v : 0.0;
      rw[ch] = ok ? w : 0.0;
    }
    double carry = 0.0;
#pragma unroll
    for (int ch = 0; ch < kScanChunks; ch++) {
      double a = rp[ch], bb = rq[ch];
      affine_scan_up(a, bb, lane);
      const double Y = fma(a, carry, bb);
      double prev = __shfl_up(Y, 1, kWave);
      if (lane == 0) prev = carry;
      ry[ch] = prev;
      carry = lane_value(Y, kWave - 1);
    }
    carry = 0.0;
#pragma unroll
    for (int ch = kScanChunks - 1; ch >= 0; ch--) {
      double a = ru[ch], bb = fma(rv[ch], ry[ch], rw[ch]);
      affine_scan_down(a, bb, lane);
      const double X = fma(a, carry, bb);
      double next = __shfl_down(X, 1, kWave);
      if (lane == kWave - 1) next = carry;
      const int r = first + ch * kWave + lane;
      if (r < first + count) {
        const long ri = (rb + r) * I.L + sl;
        gp(I.RY)[ri] = ry[ch];
        gp(I.RX)[ri] = next;
      }
      carry = lane_value(X, 0);
    }
    return;
  }
  double carry = 0.0;
  for (int ch = 0; ch < nch; ch++) {
    const int r = first + ch * kWave + lane;
    const bool ok = r < first + count;
    const long ri = (rb + (ok ? r : first)) * I.L + sl;
    const double rp = gp(I.RP)[ri], rq = gp(I.RQ)[ri];
    double a = ok ? rp : 1.0;
    double bb = ok ? rq : 0.0;
    affine_scan_up(a, bb, lane);
    const double Y = fma(a, carry, bb);
    double prev = __shfl_up(Y, 1, kWave);
    if (lane == 0) prev = carry;
    if (ok) gp(I.RY)[ri] = prev;
    carry = lane_value(Y, kWave - 1);
  }
  carry = 0.0;
  for (int ch = nch - 1; ch >= 0; ch--) {
    const int r = first + ch * kWave + lane;
    const bool ok = r < first + count;
    const long ri = (rb + (ok ? r : first)) * I.L + sl;
    const double ru = gp(I.RU)[ri], rv = gp(I.RV)[ri], rw = gp(I.RW)[ri], ry = gp(I.RY)[ri];
    double a = ok ? ru : 0.0;
    double bb = ok ? fma(rv, ry, rw) : 0.0;
    affine_scan_down(a, bb, lane);
    const double X = fma(a, carry, bb);
    double next = __shfl_down(X, 1, kWave);
    if (lane == kWave - 1) next = carry;
    if (ok) gp(I.RX)[ri] = next;
    carry = lane_value(X, 0);
  }
}

// ------------------------------------------------------------- phase 3 ---
// (single state, below: x = z + chi Yin + phi Xin in place; the slice-
// interleaved workspace defers the correction to the next load of each node)

// Single state (L = 1): one workgroup per run, kDDSeg lanes per segment, lane =
// node. The zero-carry segment solve is one forward and one backward affine
// scan across those lanes; then one lane chains the run's segments (run maps and
// the slice parts of the segments' carries, as k_dd_local_run does per slice).
constexpr int kRun1Threads = kDDRun / kSegsPerWave * kWave;
static_assert(kDDRun % kSegsPerWave == 0, "a run is a whole number of waves");

__global__ __launch_bounds__(kRun1Threads) void k_dd_local_run1(const DDInst* __restrict__ insts,
                                                                DDFactors f, int colour,
                                                                int run_begin) {
  __shared__ double sYb[kDDRun], sZa[kDDRun];
  __shared__ double sF[4][kDDRun];  // the run's PSIE, CHIA, PHIA, SA
  const DDInst& I = insts[0];
  const int ri = run_begin + blockIdx.x;
  const DDRunRec* rec = I.run_recs + ri;
  const int rlen = rec->len, seg0 = rec->seg0;  // workgroup-uniform
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int gl = lane % kDDSeg;  // node within the segment
  const int t = wv * kSegsPerWave + lane / kDDSeg;  // segment within the run
  const int slo = rec->lo[t], scnt = rec->cnt[t];  // cnt = 0 past the run's end
  const bool ok = gl < scnt;
  const long node = slo + (ok ? gl : 0);
  const long cb = (long)colour * I.n;
  const double em = gp(f.G)[cb + (node > 0 ? node - 1 : 0)];
  const double e = node > 0 ? em : 0.0;  // e = g of the previous node
  const double r = gp(f.R)[cb + node], g = gp(f.G)[cb + node];
  const double z0 = gp(I.Z)[node];
  if (threadIdx.x < 4 * kDDRun) {
    const int k = threadIdx.x / kDDRun, q = threadIdx.x - k * kDDRun;
    const int sq = seg0 + (q < rlen ? q : 0);
    const gdouble* src = gp(k == 0 ? f.PSIE : (k == 1 ? f.CHIA : (k == 2 ? f.PHIA : f.SA)));
    sF[k][q] = src[sq];
  }
  // forward: y_t = e_t y_{t-1} + d_t from y = 0 before the segment (e = 1,
  // d = 0 past its end)
  double a = ok ? e : 1.0, bb = ok ? z0 : 0.0;
  group_scan_up<kDDSeg>(a, bb, gl);
  const double y = bb;
  // backward: z_t = g_t z_{t+1} + r_t y_t from z = 0 after the segment
  a = ok ? g : 0.0;
  bb = ok ? r * y : 0.0;
  group_scan_down<kDDSeg>(a, bb, gl);
  const double z = bb;
  if (ok) gp(I.Z)[node] = z;
  const double ylast = __shfl(y, (scnt > 0 ? scnt : 1) - 1, kDDSeg);
  const double zfirst = __shfl(z, 0, kDDSeg);
  if (gl == 0) {
    sYb[t] = ylast;
    sZa[t] = zfirst;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // forward: Y before segment q = A_q Y_before + B_q; backward: X after it =
    // C_q X_after + D_q Y_before + E_q (B, E are the slice parts)
    double A = 1.0, Bq = 0.0;
    for (int q = 0; q < rlen; q++) {
      const double yb = sYb[q];
      sYb[q] = Bq;
      gp(I.Yp)[seg0 + q] = Bq;
      Bq = fma(sF[0][q], Bq, yb);
      A = sF[0][q] * A;
    }
    double C = 1.0, D = 0.0, E = 0.0;
    for (int q = rlen - 1; q >= 0; q--) {
      const double pa = sF[2][q], ca = sF[1][q];
      gp(I.Xp)[seg0 + q] = E;
      E = fma(pa, E, fma(ca, sYb[q], sZa[q]));
      D = fma(pa, D, ca * sF[3][q]);
      C = pa * C;
    }
    gp(I.RP)[ri] = A;
    gp(I.RQ)[ri] = Bq;
    gp(I.RU)[ri] = C;
    gp(I.RV)[ri] = D;
    gp(I.RW)[ri] = E;
  }
}

__global__ __launch_bounds__(4 * kWave) void k_dd_correct1(const DDInst* __restrict__ insts,
                                                           DDFactors f, int colour,
                                                           int seg_begin, int seg_count) {
  const DDInst& I = insts[0];
  const int lane = threadIdx.x & (kWave - 1);
  const int gl = lane % kDDSeg;
  const int w = (int)(blockIdx.x * 4 + threadIdx.x / kWave) * kSegsPerWave + lane / kDDSeg;
  if (w >= seg_count) return;
  const int si = seg_begin + w;
  const DDSeg sg = I.segs[si];
  if (gl >= sg.len) return;
  const long node = sg.lo + gl;
  const long cb = (long)colour * I.n;
  // the segment's carries from its run's carries and its slice parts
  const int r = I.seg_run[si];
  const double ry = gp(I.RY)[r], rx = gp(I.RX)[r];
  const double yin = fma(gp(f.SA)[si], ry, gp(I.Yp)[si]);
  const double xin = fma(gp(f.SC)[si], rx, fma(gp(f.SD)[si], ry, gp(I.Xp)[si]));
  gp(I.Z)[node] =
      fma(gp(f.PHI)[cb + node], xin, fma(gp(f.CHI)[cb + node], yin, gp(I.Z)[node]));
}

// ------------------------------------------------------ parareal update ---
// Whole-state update; the block's largest |change| (mode 1) goes to
// partial[block] (plain read-modify-write: launches run in stream order).
__global__ __launch_bounds__(256) void k_update(const double* __restrict__ g,
                                                const double* __restrict__ F,
                                                double* __restrict__ Gold,
                                                double* __restrict__ Unext, size_t n, int mode,
                                                unsigned long long* __restrict__ partial) {
  __shared__ unsigned long long wm[4];
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  unsigned long long mx = 0;
  for (; i < n; i += stride) {
    const double gv = g[i];
    if (mode == 2) {
      Unext[i] = gv;
    } else {
      const double un = F[i] + (gv - Gold[i]);
      const unsigned long long bits = abs_bits(un - Unext[i]);
      mx = bits > mx ? bits : mx;
      Unext[i] = un;
    }
    Gold[i] = gv;
  }
  if (mode == 1) {
    for (int off = 32; off > 0; off >>= 1) {
      unsigned long long o = __shfl_xor(mx, off, kWave);
      mx = o > mx ? o : mx;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) wm[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < 4; w++) mx = wm[w] > mx ? wm[w] : mx;
      if (mx > partial[blockIdx.x]) partial[blockIdx.x] = mx;
    }
  }
}

}  // namespace

hipError_t launch_dd_faces(const double* rho, const double* a, int n, int n_colors, double* w,
                           hipStream_t s) {
  long total = (long)(n + 1) * n_colors;
  hipLaunchKernelGGL(k_dd_faces, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, rho, a, n,
                     n_colors, w);
  return hipGetLastError();
}

hipError_t launch_dd_factorize(const double* w, int n, const int* comp_lo, const int* comp_hi,
                               const int* comp_colour, int n_comps, double tau_over_h2, double* R,
                               double* G, hipStream_t s) {
  hipLaunchKernelGGL(k_dd_factorize, dim3((n_comps + 63) / 64), dim3(64), 0, s, w, n, comp_lo,
                     comp_hi, comp_colour, n_comps, tau_over_h2, R, G);
  return hipGetLastError();
}

hipError_t launch_dd_segfactors(const DDSeg* segs, const int* seg_colour, int n_segs, int n,
                                const double* R, const double* G, double* CHI,
                                double* PHI, double* PSIE, double* CHIA, double* PHIA,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_dd_segfactors, dim3((n_segs + 63) / 64), dim3(64), 0, s, segs, seg_colour,
                     n_segs, n, R, G, CHI, PHI, PSIE, CHIA, PHIA);
  return hipGetLastError();
}

template <int L>
static hipError_t dd_local_run_t(const DDInst* d, const DDInst& h, const DDFactors& f, int colour,
                                 int run_begin, int run_count, bool stale_ok, hipStream_t s) {
  dim3 grid(run_count, h.B);
  hipLaunchKernelGGL((k_dd_local_run<L>), grid, dim3(kDDRun * L), 0, s, d, f, colour, run_begin,
                     (int)stale_ok);
  return hipGetLastError();
}

hipError_t launch_dd_local(const DDInst* d, const DDInst& h, const DDFactors& f, int colour,
                           int seg_begin, int seg_count, int run_begin, int run_count,
                           bool stale_ok, hipStream_t s) {
  if (run_count <= 0) return hipSuccess;
  if (h.L == 1) {
    hipLaunchKernelGGL(k_dd_local_run1, dim3(run_count), dim3(kRun1Threads), 0, s, d, f, colour,
                       run_begin);
    return hipGetLastError();
  }
  switch (h.L) {
    case 8: return dd_local_run_t<8>(d, h, f, colour, run_begin, run_count, stale_ok, s);
    case 16: return dd_local_run_t<16>(d, h, f, colour, run_begin, run_count, stale_ok, s);
    case 32: return dd_local_run_t<32>(d, h, f, colour, run_begin, run_count, stale_ok, s);
    case 64: return dd_local_run_t<64>(d, h, f, colour, run_begin, run_count, stale_ok, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_dd_runfactors(const DDInst* d, const DDInst& h, const DDFactors& f, double* SA,
                                double* SC, double* SD, hipStream_t s) {
  if (h.n_runs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dd_runfactors, dim3((h.n_runs + 127) / 128), dim3(128), 0, s, d, f, SA, SC,
                     SD);
  return hipGetLastError();
}

hipError_t launch_dd_pending(const DDInst* d, const DDInst& h, const DDFactors& f, double* PC0,
                             double* PP0, double* PC1, double* PP1, double* FC, double* FP,
                             hipStream_t s) {
  const long total = (long)h.n_segs * kDDSeg + h.n;
  hipLaunchKernelGGL(k_dd_pending, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, d, f,
                     PC0, PP0, PC1, PP1, FC, FP);
  return hipGetLastError();
}

hipError_t launch_dd_from_interleaved(const DDInst* d, const DDInst& h, const DDFactors& f,
                                      double* F, hipStream_t s) {
  const long total = (long)h.B * h.n_segs * h.L;
  if (total > 0)
    hipLaunchKernelGGL(k_dd_final_carries, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       d, f);
  hipLaunchKernelGGL(k_dd_from_interleaved, dim3((h.n + 63) / 64, h.B), dim3(4 * kWave), 0, s, d,
                     f, F);
  return hipGetLastError();
}

hipError_t launch_dd_carries(const DDInst* d, const DDInst& h, const DDFactors& f, int run_begin,
                             int run_count, const int* comp_run_first, const int* comp_run_count,
                             int n_comps, hipStream_t s) {
  if (n_comps <= 0 || run_count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dd_runscan, dim3(n_comps, h.B * h.L), dim3(kWave), 0, s, d, comp_run_first,
                     comp_run_count);
  return hipGetLastError();
}

hipError_t launch_dd_correct(const DDInst* d, const DDInst& h, const DDFactors& f, int colour,
                             int seg_begin, int seg_count, hipStream_t s) {
  if (seg_count <= 0) return hipSuccess;
  if (h.L != 1) return hipErrorInvalidValue;  // the interleaved workspace defers it
  hipLaunchKernelGGL(k_dd_correct1, dim3((seg_count + 4 * kSegsPerWave - 1) / (4 * kSegsPerWave)),
                     dim3(4 * kWave), 0, s, d, f, colour, seg_begin, seg_count);
  return hipGetLastError();
}

int update_blocks(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 2048); }

hipError_t launch_update(const double* g, const double* F, double* G_old, double* U_next,
                         size_t n, int mode, unsigned long long* partial, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_update, dim3(update_blocks(n)), dim3(256), 0, s, g, F, G_old, U_next, n,
                     mode, partial);
  return hipGetLastError();
}

}  // namespace prk
