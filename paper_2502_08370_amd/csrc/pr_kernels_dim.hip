// HIP kernels (gfx950, wave64, FP64) for the dimensional-splitting FIE
// propagators of parareal with splitting (arXiv 2502.08370, section 2.2
// eq. FIE_method; section 3 for the propagators and the parareal update).
//
// Every substep (I - tau A_dir) V = U is a set of independent tridiagonal
// line solves (section 2.2, last paragraphs). The matrices do not change in
// time, so each line's LU factorisation is computed once per tau and reused
// by every slice and every step.
#include "pr_internal.h"

namespace prk {

namespace {

constexpr int kWave = 64;

#define GLOBAL __attribute__((address_space(1)))
typedef GLOBAL double gdouble;
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef GLOBAL dv2 gdv2;

// Pointers read from descriptor tables are generic; these casts let the
// compiler emit global (not flat) memory instructions for them.
__device__ __forceinline__ gdouble* gp(double* p) { return (gdouble*)p; }
__device__ __forceinline__ const gdouble* gp(const double* p) { return (const gdouble*)p; }

__device__ __forceinline__ unsigned long long abs_bits(double v) {
  return static_cast<unsigned long long>(__double_as_longlong(fabs(v)));
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// Value of v held by lane `src` (wave-uniform result).
__device__ __forceinline__ double lane_value(double v, int src) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Inclusive scan over the 64 lanes, in lane order, of the affine maps
// y -> a*y + b: lane i ends with the composition f_i o ... o f_0.
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

// Same in reverse lane order: lane i ends with f_i o f_{i+1} o ... o f_63.
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

// ---------------------------------------------------------------- setup ---

// Face coefficient = mean of e^theta over the face's two nodes; theta is
// nodal on the extended (ny+2) x (nx+2) grid.
__global__ void k_faces_from_theta_2d(const double* __restrict__ theta, int nx, int ny,
                                      double* __restrict__ ax, double* __restrict__ ay) {
  const long W = nx + 2;
  const long nax = (long)ny * (nx + 1), nay = (long)(ny + 1) * nx;
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < nax) {
    long j = t / (nx + 1), f = t % (nx + 1);
    double tp = theta[(j + 1) * W + f], tq = theta[(j + 1) * W + f + 1];
    ax[t] = 0.5 * (exp(tp) + exp(tq));
  } else if (t < nax + nay) {
    long u = t - nax;
    long g = u / nx, i = u % nx;
    double tp = theta[g * W + i + 1], tq = theta[(g + 1) * W + i + 1];
    ay[u] = 0.5 * (exp(tp) + exp(tq));
  }
}

__global__ void k_faces_from_theta_1d(const double* __restrict__ theta, int nx,
                                      double* __restrict__ ax) {
  long f = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (f <= nx) ax[f] = 0.5 * (exp(theta[f]) + exp(theta[f + 1]));
}

// LU factorisation of I - tau A along each line (one thread per line). Row p:
// -w_p x_{p-1} + (1 + w_p + w_{p+1} + react) x_p - w_{p+1} x_{p+1}.
__global__ void k_factorize(FactorJob job) {
  int line = blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= job.n_lines) return;
  const double* face = job.face + line * job.face_line_stride;
  // the matrix is symmetric, so the forward multiplier e_p = w_p / u_{p-1}
  // equals the previous back-substitution factor g_{p-1} = w_p r_{p-1}; both
  // are formed as that product so that E[p] == G[p-1] exactly
  double r_prev = 0.0;
  double wl = job.tau_over_h2 * face[0];
  for (int p = 0; p < job.n_pos; p++) {
    double wr = job.tau_over_h2 * face[(long)(p + 1) * job.face_pos_stride];
    double diag = 1.0 + wl + wr + job.react;
    double e = (p == 0) ? 0.0 : wl * r_prev;
    double u = diag - wl * e;
    double r = 1.0 / u;
    double g = (p + 1 < job.n_pos) ? wr * r : 0.0;
    long idx = job.pos_major ? (long)p * job.n_lines + line : (long)line * job.n_pos + p;
    if (job.E) job.E[idx] = e;
    job.R[idx] = r;
    job.G[idx] = g;
    r_prev = r;
    wl = wr;
  }
}

// phi_p = prod_{t=p..chunk end} g_t for chunks of M positions (line-major G);
// phiC position-major [p][line], phiS[line][k] = phi at the chunk's first position.
__global__ void k_chunk_phi(const double* __restrict__ G, int n_lines, int n_pos, int M,
                            double* __restrict__ phiC, double* __restrict__ phiS) {
  int line = blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= n_lines) return;
  const int P = (n_pos + M - 1) / M;
  for (int k = 0; k < P; k++) {
    int p0 = k * M, p1 = min(n_pos, p0 + M);
    double phi = 1.0;
    for (int p = p1 - 1; p >= p0; p--) {
      phi = G[(long)line * n_pos + p] * phi;
      phiC[(long)p * n_lines + line] = phi;
    }
    phiS[(long)line * P + k] = phi;
  }
}

// Twisted factorisation of I - tau A along each line (one thread per line):
// positions p < mid keep the LU factors of k_factorize (the top part does not
// depend on the rest of the line); positions p >= mid get the UL factors of
// the bottom part, eliminated from the line end: v_{n-1} = diag, v_p = diag_p -
// w_{p+1}^2 / v_{p+1}, r_p = 1 / v_p, g_p = w_p r_p (coupling to p - 1, so the
// upward multiplier e_p = w_{p+1} / v_{p+1} is g_{p+1} exactly).
__global__ void k_factorize_twisted(FactorJob job, int mid) {
  int line = blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= job.n_lines) return;
  const double* face = job.face + line * job.face_line_stride;
  const int n = job.n_pos;
  const int m = min(mid, n);
  double r_prev = 0.0;
  double wl = job.tau_over_h2 * face[0];
  for (int p = 0; p < m; p++) {
    double wr = job.tau_over_h2 * face[(long)(p + 1) * job.face_pos_stride];
    double diag = 1.0 + wl + wr + job.react;
    double e = (p == 0) ? 0.0 : wl * r_prev;
    double u = diag - wl * e;
    double r = 1.0 / u;
    double g = (p + 1 < n) ? wr * r : 0.0;
    long idx = (long)line * n + p;
    job.R[idx] = r;
    job.G[idx] = g;
    r_prev = r;
    wl = wr;
  }
  double r_next = 0.0;
  double wr = job.tau_over_h2 * face[(long)n * job.face_pos_stride];
  for (int p = n - 1; p >= m; p--) {
    double wlp = job.tau_over_h2 * face[(long)p * job.face_pos_stride];
    double diag = 1.0 + wlp + wr + job.react;
    double e = (p == n - 1) ? 0.0 : wr * r_next;
    double v = diag - wr * e;
    double r = 1.0 / v;
    double g = (p > 0) ? wlp * r : 0.0;
    long idx = (long)line * n + p;
    job.R[idx] = r;
    job.G[idx] = g;
    r_next = r;
    wr = wlp;
  }
}

// phi of the twisted factorisation: chunks k < kmid as k_chunk_phi (product of g
// from the position to the chunk end), chunks k >= kmid from the chunk start to
// the position; phiS[line][k] = the product over the whole chunk.
__global__ void k_chunk_phi_twisted(const double* __restrict__ G, int n_lines, int n_pos, int M,
                                    int kmid, double* __restrict__ phiC,
                                    double* __restrict__ phiS) {
  int line = blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= n_lines) return;
  const int P = (n_pos + M - 1) / M;
  for (int k = 0; k < P; k++) {
    int p0 = k * M, p1 = min(n_pos, p0 + M);
    double phi = 1.0;
    if (k < kmid) {
      for (int p = p1 - 1; p >= p0; p--) {
        phi = G[(long)line * n_pos + p] * phi;
        phiC[(long)p * n_lines + line] = phi;
      }
    } else {
      for (int p = p0; p < p1; p++) {
        phi = G[(long)line * n_pos + p] * phi;
        phiC[(long)p * n_lines + line] = phi;
      }
    }
    phiS[(long)line * P + k] = phi;
  }
}

__global__ void k_interleave_pairs(const double* __restrict__ a, const double* __restrict__ b, long n,
                                   double* __restrict__ out) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p < n) {
    out[2 * p] = a[p];
    out[2 * p + 1] = b[p];
  }
}

// ------------------------------------------------- interleave transposes ---

// Natural U[slice][j][i] <-> Z[b][j][i][l] through a 64 x 64 LDS tile; one
// block of kTrWaves waves per (64-column tile, row, slice block). Every load of
// a thread is issued before its first LDS store.
constexpr int kTrWaves = 4;
constexpr int kTrThreads = kTrWaves * kWave;
constexpr int kTrIt = kWave * kWave / kTrThreads;  // tile entries per thread

__global__ __launch_bounds__(kTrThreads) void k_to_interleaved(const DimInst* __restrict__ insts,
                                                               const double* __restrict__ U) {
  __shared__ double tile[64][65];
  const DimInst& I = insts[0];
  if (I.active && !I.active[I.idx]) return;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int i0 = blockIdx.x * 64, j = blockIdx.y, b = blockIdx.z;
  const int L = I.L, nx = I.nx, lg = 31 - __clz(L);
  const long slab = I.slab;
  const long npts = (long)nx * I.ny;
  const int i = i0 + lane;
  double v[kTrIt];
#pragma unroll
  for (int u = 0; u < kTrIt; u++) {
    const int sl = w + kTrWaves * u, slice = b * L + sl;
    v[u] = (sl < L && slice < I.N && i < nx) ? U[slice * npts + (long)j * nx + i] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kTrIt; u++) {
    const int sl = w + kTrWaves * u;
    if (sl < L) tile[sl][lane] = v[u];
  }
  __syncthreads();
  gdouble* Zb = gp(I.Z) + b * slab + ((long)j * nx + i0) * L;
  const int n = min(64, nx - i0) * L;
#pragma unroll
  for (int u = 0; u < kTrIt; u++) {
    const int q = tid + kTrThreads * u;
    if (q < n) Zb[q] = tile[q & (L - 1)][q >> lg];
  }
}

// Z (+ the pending chunk correction of the last y sweep) -> natural F[slice][j][i].
__global__ __launch_bounds__(kTrThreads) void k_from_interleaved(
    const DimInst* __restrict__ insts, double* __restrict__ F, int with_corr) {
  __shared__ double tile[64][65];
  const DimInst& I = insts[0];
  if (I.active && !I.active[I.idx]) return;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int i0 = blockIdx.x * 64, j = blockIdx.y, b = blockIdx.z;
  const int L = I.L, nx = I.nx, M = I.M, Py = I.Py, lg = 31 - __clz(L);
  const long npts = (long)nx * I.ny;
  const gdouble* Zb = gp(I.Z) + b * I.slab + ((long)j * nx + i0) * L;
  const gdouble* sig = with_corr ? gp(I.sigY) + ((long)b * Py + j / M) * nx * L : nullptr;
  const gdouble* phiC = with_corr ? gp(I.fyPhiC) + (long)j * nx : nullptr;
  const int n = min(64, nx - i0) * L;
  double z[kTrIt], ph[kTrIt], sg[kTrIt];
#pragma unroll
  for (int u = 0; u < kTrIt; u++) {
    const int q = tid + kTrThreads * u;
    const bool ok = q < n;
    const int t = q >> lg, sl = q & (L - 1);
    z[u] = ok ? Zb[q] : 0.0;
    ph[u] = (ok && with_corr) ? phiC[i0 + t] : 0.0;
    sg[u] = (ok && with_corr) ? sig[(long)(i0 + t) * L + sl] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kTrIt; u++) {
    const int q = tid + kTrThreads * u;
    if (q < n) tile[q & (L - 1)][q >> lg] = fma(ph[u], sg[u], z[u]);
  }
  __syncthreads();
  const int cnt = min(64, nx - i0);
#pragma unroll
  for (int u = 0; u < kTrIt; u++) {
    const int sl = w + kTrWaves * u, slice = b * L + sl;
    if (sl < L && slice < I.N && lane < cnt)
      F[slice * npts + (long)j * nx + i0 + lane] = tile[sl][lane];
  }
}

// Natural U[slice][node] <-> the partitioned sweeps' blocks Z[b][node][l] (Lp
// slices per block, not a power of two). Into the blocks: a workgroup stages 64
// nodes of the block's slices in LDS, reading each slice's 64 nodes as one run
// and writing the 64 * Lp doubles of the block as one run. Back: one thread per
// (node, block) reads its node's run and writes the node in each slice, 64
// consecutive nodes per wave.
constexpr int kPartTrNodes = 64;
__global__ __launch_bounds__(256) void k_to_part(const DimInst* __restrict__ insts,
                                                 const double* __restrict__ U) {
  __shared__ double tile[kPartTrNodes * kWave];
  const DimInst& I = insts[0];
  if (I.active && !I.active[I.idx]) return;
  const long npts = (long)I.nx * I.ny;
  const long n0 = (long)blockIdx.x * kPartTrNodes;
  const int b = blockIdx.y, L = I.Lp, nb = min(L, I.N - b * L);
  const int cnt = (int)min((long)kPartTrNodes, npts - n0);
  const gdouble* u = gp(U) + (long)b * L * npts + n0;
  constexpr int kIt = kPartTrNodes * kWave / 256;  // entries per thread at most
  double v[kIt];
#pragma unroll
  for (int k = 0; k < kIt; k++) {  // every load issued before the first LDS store
    const int e = threadIdx.x + 256 * k, l = e / kPartTrNodes, nd = e - l * kPartTrNodes;
    v[k] = (l < nb && nd < cnt) ? u[(long)l * npts + nd] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < kIt; k++) {
    const int e = threadIdx.x + 256 * k, l = e / kPartTrNodes, nd = e - l * kPartTrNodes;
    if (l < L) tile[nd * L + l] = v[k];
  }
  __syncthreads();
  gdouble* z = gp(I.Z) + b * I.slabp + n0 * L;
  for (int e = threadIdx.x; e < cnt * L; e += blockDim.x) z[e] = tile[e];
}

__global__ __launch_bounds__(256) void k_from_part(const DimInst* __restrict__ insts,
                                                   double* __restrict__ F) {
  const DimInst& I = insts[0];
  if (I.active && !I.active[I.idx]) return;
  const long npts = (long)I.nx * I.ny;
  const long node = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int b = blockIdx.y, L = I.Lp, nb = min(L, I.N - b * L);
  if (node >= npts) return;
  const gdouble* z = gp(I.Z) + b * I.slabp + node * L;
  gdouble* f = gp(F) + (long)b * L * npts + node;
  for (int l0 = 0; l0 < nb; l0 += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; k++) v[k] = l0 + k < nb ? z[l0 + k] : 0.0;
#pragma unroll
    for (int k = 0; k < 8; k++)
      if (l0 + k < nb) f[(long)(l0 + k) * npts] = v[k];
  }
}

// -------------------------------------------------------- fine sweeps ---

// One substep of the fine FIE step for every line of direction DIR of every
// slice of the work items' instances. Lanes = (line in group, slice); each
// wave walks its lines in chunks of M positions, holding one chunk in
// registers while the next one is being loaded. With HP, the pending chunk
// correction of the previous (other-direction) sweep is added on load.
// A partial last chunk is computed in full on clamped loads: the multiplier
// that couples the line's last position to the next one is 0 (stored so for
// the top part, forced for the bottom part), so the padded positions cannot
// leak into the real ones, and only real positions are stored. The workspace values are
// written with nontemporal stores (each is read once, by the next sweep), which
// keeps the reused carries and factors in the caches.
//
// TW (twisted factorisation): a workgroup of two waves per line group, which
// doubles the waves in flight without adding registers per wave. The first
// wave takes the chunks [0, kmid) with the LU factors of the line's top part
// (forward y_p = d_p + g_{p-1} y_{p-1}; chunk-local back substitution
// z_p = r_p y_p + g_p z_{p+1}, zero past the chunk end); the second wave the
// chunks [kmid, P) from the bottom with the UL factors stored at those
// positions (upward y_p = d_p + g_{p+1} y_{p+1}; chunk-local substitution
// z_p = r_p y_p + g_p z_{p-1}, zero before the chunk start). At mid = kmid*M
// the true values follow from the two innermost chunk-local values:
// x_{mid-1} = z_{mid-1} + g_{mid-1} x_mid and x_mid = z_mid + g_mid x_{mid-1}.
// Each wave then resolves its chunks' carries outwards. The consumer's
// correction keeps its form x_p = z_p + phi_p sigma_k: for a bottom chunk phi
// is the product of its g from the chunk start to p and sigma the true value
// just before the chunk.
template <int L, int M, int DIR, bool HP, int SGN = 0, bool FT = false, bool TW = false>
__global__ __launch_bounds__(TW ? 2 * kWave : kWave) void k_fine_sweep(
    const DimInst* __restrict__ insts, const WorkItem* __restrict__ work, int step) {
  constexpr int G = kWave / L;  // lines per wave
  constexpr bool kUni = (L == kWave);
  constexpr int NQ = kUni ? 1 : (G * M + kWave - 1) / kWave;
  // per-position rows: e, r, g, phi of the pending correction, and with a
  // source the spatial factors S_0, S_1
  constexpr int NF = FT ? 4 + kMaxForcing : 4;
  constexpr int NW = TW ? 2 : 1;  // waves per workgroup
  static_assert(M <= kWave, "chunk longer than a wave");
  static_assert(!FT || DIR == 0, "the source enters the first (x) stage");
  // factor staging when a wave holds several lines: [wave][NF][G][M+1]
  __shared__ double sF[NW][kUni ? 1 : NF][kUni ? 1 : G][M + 1];
  // outer chunk-local value of every chunk of the group's lines (the first of a
  // top chunk, the last of a bottom chunk), resolved into carries at the end;
  // lines of more chunks park them in the carry slots they resolve into
  constexpr int kMaxChunks = (kLineSeg + M - 1) / M;
  __shared__ double zouter[kMaxChunks][kWave];
  __shared__ double zmid[NW][kWave];  // innermost chunk-local values of the two waves

  const WorkItem w = work[blockIdx.x];
  const DimInst& I = insts[w.inst];
  if (step >= I.steps) return;  // this instance has finished its fine steps
  if (I.active && !I.active[I.idx]) return;  // converged instance
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = TW ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;
  const int gsub = lane / L;
  const int sl = lane - gsub * L;

  const int n_lines = DIR == 0 ? I.ny : I.nx;
  const int n_pos = DIR == 0 ? I.nx : I.ny;
  const int P = DIR == 0 ? I.Px : I.Py;
  // chunks [kbeg, kend) of this wave; the bottom part starts at chunk kmid
  const int kmid = TW ? min(DIR == 0 ? I.twx : I.twy, P) : P;
  const bool bottom = TW && wv == 1;
  const int kbeg = bottom ? kmid : 0, kend = bottom ? P : kmid;
  const int nl_prev = n_pos;  // lines of the previous sweep = our positions
  const long pstr = DIR == 0 ? (long)L : (long)I.nx * L;
  const long lstr = DIR == 0 ? (long)I.nx * L : (long)L;
  const gdouble* R = gp(DIR == 0 ? I.fxR : I.fyR);
  const gdouble* Gf = gp(DIR == 0 ? I.fxG : I.fyG);
  const gdouble* phiS = gp(DIR == 0 ? I.fxPhiS : I.fyPhiS);
  const gdouble* phiPrev = gp(DIR == 0 ? I.fyPhiC : I.fxPhiC);
  const gdouble* sigPrev = DIR == 0 ? gp(I.sigY) + (long)w.b * I.Py * I.nx * L
                                    : gp(I.sigX) + (long)w.b * I.Px * I.ny * L;
  gdouble* sigOut = DIR == 0 ? gp(I.sigX) + (long)w.b * I.Px * I.ny * L
                             : gp(I.sigY) + (long)w.b * I.Py * I.nx * L;

  const int line0 = w.group * G;
  const int line = line0 + gsub;
  const bool active = line < n_lines;
  const int lc = active ? line : n_lines - 1;  // clamped for in-bounds loads
  // chunk outer values in LDS, or (longer lines) in this lane's carry slots:
  // a top chunk's in the slot of the chunk above it, a bottom chunk's in the
  // slot of the chunk below it, which the resolution reads before overwriting
  const bool zlds = P <= kMaxChunks;  // wave-uniform
  gdouble* zslot = sigOut + (long)lc * L + sl;
  const long kstr = (long)n_lines * L;
  // row of the previous sweep's carries for the chunk that holds this line
  const gdouble* sgRow = sigPrev + ((long)(lc / M) * nl_prev) * L + sl;
  gdouble* zbase = gp(I.Z) + w.b * I.slab + (long)lc * lstr + sl;
  const long frow = (long)line0 * n_pos;  // line-uniform factor row when kUni

  // With one line per wave the row pointers are wave-uniform: keep them apart
  // from the per-lane slice offset so addresses are scalar base + lane offset.
  const gdouble* zrow_u = gp(I.Z) + w.b * I.slab + (long)line0 * lstr;
  const gdouble* sgrow_u = sigPrev + ((long)(line0 / M) * nl_prev) * L;
  const unsigned usl = (unsigned)sl;  // lane offset (unsigned: scalar-base addressing)
  // DR: the stencil array lives at the same offsets as Z; its values are held
  // in their own registers (sv) and combined when the chunk is processed
  const long drOff = SGN != 0 ? (long)(I.drS - I.Z) : 0;
  constexpr int MS = SGN != 0 ? M : 1;
  const long zo = I.zout;  // stores go to Z + zout (out-of-place recompute of the adjoint)
  // source: dt * g_m of this lane's slice at this step (0 on padding slices)
  double gl[kMaxForcing] = {};
  const gdouble* fS = FT ? gp(I.fS) : nullptr;
  if constexpr (FT) {
    const int slice = w.b * L + sl;
    const long nst = (long)I.N * I.steps;
    const long gi = (long)(slice < I.N ? slice : 0) * I.steps + step;
#pragma unroll
    for (int m = 0; m < kMaxForcing; m++) {
      const double g = gp(I.fgf)[m * nst + gi];
      gl[m] = slice < I.N ? g : 0.0;
    }
  }
  auto issue = [&](double (&v)[M], double (&sv)[MS], double (&sg)[M], double (&f)[NF][NQ],
                   int k) {
    const int p0 = k * M;
    const int cnt = min(M, n_pos - p0);
    // factors first: a wait for an older load is a wait for everything issued
    // before it, and the factor registers are the first to be reused
    if constexpr (kUni) {
      // lanes past the line end load clamped entries (their values are not used
      // for the real positions; see process_up for the one multiplier that is)
      const long idx = frow + p0 + (lane < cnt ? lane : 0);
      f[1][0] = R[idx];
      f[2][0] = Gf[idx];
      if constexpr (HP) f[3][0] = phiPrev[idx];
      if constexpr (FT) {
#pragma unroll
        for (int m = 0; m < kMaxForcing; m++) f[4 + m][0] = fS[m * I.npts + idx];
      }
    } else {
#pragma unroll
      for (int qq = 0; qq < NQ; qq++) {
        const int q = lane + qq * kWave;
        const int g = q / M, t = q - g * M;
        const int ln = line0 + g, p = p0 + t;
        const bool ok = q < G * M && ln < n_lines && p < n_pos;
        const long idx = ok ? (long)ln * n_pos + p : 0;
        // e_p: g_{p-1} eliminating downwards (top), g_{p+1} upwards (bottom)
        if (bottom)
          f[0][qq] = (ok && p + 1 < n_pos) ? Gf[idx + 1] : 0.0;
        else
          f[0][qq] = (ok && p > 0) ? Gf[idx - 1] : 0.0;
        f[1][qq] = R[idx];
        f[2][qq] = Gf[idx];
        if constexpr (HP) f[3][qq] = phiPrev[idx];
        if constexpr (FT) {
#pragma unroll
          for (int m = 0; m < kMaxForcing; m++) f[4 + m][qq] = fS[m * I.npts + idx];
        }
      }
    }
    if constexpr (kUni) {
      const gdouble* zc = zrow_u + (long)p0 * pstr;
      const gdouble* sc = sgrow_u + (long)p0 * L;
#pragma unroll
      for (int t = 0; t < M; t++) {
        const int tt = (cnt == M || t < cnt) ? t : 0;
        v[t] = (zc + (long)tt * pstr)[usl];
        if constexpr (SGN != 0) sv[t] = (zc + drOff + (long)tt * pstr)[usl];
        if constexpr (HP) sg[t] = (sc + (long)tt * L)[usl];
      }
    } else {
      const gdouble* zc = zbase + (long)p0 * pstr;
      const gdouble* sc = sgRow + (long)p0 * L;
      if (cnt == M) {
#pragma unroll
        for (int t = 0; t < M; t++) {
          v[t] = zc[t * pstr];
          if constexpr (SGN != 0) sv[t] = zc[drOff + t * pstr];
        }
        if constexpr (HP) {
#pragma unroll
          for (int t = 0; t < M; t++) sg[t] = sc[t * L];
        }
      } else {
#pragma unroll
        for (int t = 0; t < M; t++) {
          const int tt = t < cnt ? t : 0;
          v[t] = zc[tt * pstr];
          if constexpr (SGN != 0) sv[t] = zc[drOff + tt * pstr];
          if constexpr (HP) sg[t] = sc[tt * L];
        }
      }
    }
  };

  double ycarry = 0.0;
  double gcarry = 0.0;  // kUni: e of the chunk's first processed position, from the previous chunk
  double zin = 0.0;     // chunk-local value at this wave's innermost position
  // Staging of a chunk's factor rows in LDS (several lines per wave) and the
  // per-position load corrections (pending carry, DR term, source).
  auto stage = [&](double (&f)[NF][NQ]) {
    if constexpr (!kUni) {
#pragma unroll
      for (int qq = 0; qq < NQ; qq++) {
        const int q = lane + qq * kWave;
        if (q < G * M) {
          const int g = q / M, t = q - g * M;
#pragma unroll
          for (int c = 0; c < NF; c++)
            if (HP || c != 3) sF[wv][c][g][t] = f[c][qq];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  };
  auto rhs = [&](double (&v)[M], double (&sv)[MS], double (&sg)[M], auto fac, int t) -> double {
    double d = v[t];
    if constexpr (HP) d = fma(fac(3, t), sg[t], d);
    if constexpr (SGN > 0) {
      // x stage of DR: U + S; S carries the same pending correction as U
      if constexpr (HP) sv[t] = fma(fac(3, t), sg[t], sv[t]);
      d = d + sv[t];
    } else if constexpr (SGN < 0) {
      d = d - sv[t];  // y stage: W - S
      sv[t] = d;      // kept: the next step's S is U' - (W - S)
    }
    if constexpr (FT) {
#pragma unroll
      for (int m = 0; m < kMaxForcing; m++) d = fma(gl[m], fac(4 + m, t), d);
    }
    return d;
  };
  auto store = [&](double (&v)[M], double (&sv)[MS], int k) {
    const int p0 = k * M;
    const int cnt = min(M, n_pos - p0);
    if constexpr (SGN < 0) {
#pragma unroll
      for (int t = 0; t < M; t++) sv[t] = v[t] - sv[t];  // S' = U' - Y (same pending correction)
    }
    if constexpr (kUni) {
      gdouble* zc = (gdouble*)zrow_u + (long)p0 * pstr;
      if (cnt == M) {
#pragma unroll
        for (int t = 0; t < M; t++) {
          __builtin_nontemporal_store(v[t], &(zc + zo + (long)t * pstr)[usl]);
          if constexpr (SGN != 0) __builtin_nontemporal_store(sv[t], &(zc + drOff + (long)t * pstr)[usl]);
        }
      } else {
#pragma unroll
        for (int t = 0; t < M; t++)
          if (t < cnt) {
            __builtin_nontemporal_store(v[t], &(zc + zo + (long)t * pstr)[usl]);
            if constexpr (SGN != 0) __builtin_nontemporal_store(sv[t], &(zc + drOff + (long)t * pstr)[usl]);
          }
      }
    } else if (active) {
      gdouble* zc = zbase + (long)p0 * pstr;
      if (cnt == M) {
#pragma unroll
        for (int t = 0; t < M; t++) {
          __builtin_nontemporal_store(v[t], &zc[zo + t * pstr]);
          if constexpr (SGN != 0) __builtin_nontemporal_store(sv[t], &zc[drOff + t * pstr]);
        }
      } else {
#pragma unroll
        for (int t = 0; t < M; t++)
          if (t < cnt) {
            __builtin_nontemporal_store(v[t], &zc[zo + t * pstr]);
            if constexpr (SGN != 0) __builtin_nontemporal_store(sv[t], &zc[drOff + t * pstr]);
          }
      }
    }
  };

  // top part: eliminate downwards, substitute upwards inside the chunk
  auto process_down = [&](double (&v)[M], double (&sv)[MS], double (&sg)[M],
                          double (&f)[NF][NQ], int k) {
    stage(f);
    auto fac = [&](int c, int t) -> double {
      if constexpr (kUni) {
        if (c == 0)  // e_p = g_{p-1}: the previous lane's g, or the last g of the previous chunk
          return t == 0 ? gcarry : lane_value(f[2][0], t - 1);
        return lane_value(f[c][0], t);
      } else {
        return sF[wv][c][gsub][t];
      }
    };
    double y = ycarry;
#pragma unroll
    for (int t = 0; t < M; t++) {
      const double d = rhs(v, sv, sg, fac, t);
      y = fma(fac(0, t), y, d);
      v[t] = y;
    }
    ycarry = y;
    if constexpr (kUni) gcarry = lane_value(f[2][0], M - 1);
    double z = 0.0;
#pragma unroll
    for (int t = M - 1; t >= 0; t--) {
      z = fma(fac(2, t), z, fac(1, t) * v[t]);
      v[t] = z;
    }
    zin = v[M - 1];
    store(v, sv, k);
    // resolved into the previous chunk's carry below
    if (zlds) zouter[k][lane] = v[0];
    else if (active && k > kbeg) zslot[(long)(k - 1) * kstr] = v[0];
    if constexpr (!kUni) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  };
  // bottom part (TW): eliminate upwards, substitute downwards inside the chunk
  auto process_up = [&](double (&v)[M], double (&sv)[MS], double (&sg)[M],
                        double (&f)[NF][NQ], int k) {
    stage(f);
    const int cnt = min(M, n_pos - k * M);
    auto fac = [&](int c, int t) -> double {
      if constexpr (kUni) {
        // e_p = g_{p+1}: the next lane's g, or the first g of the previous chunk;
        // 0 at the line's last position (the lanes past it hold clamped loads)
        if (c == 0)
          return t == M - 1 ? gcarry : (t + 1 < cnt ? lane_value(f[2][0], t + 1) : 0.0);
        return lane_value(f[c][0], t);
      } else {
        return sF[wv][c][gsub][t];
      }
    };
    double y = ycarry;
#pragma unroll
    for (int t = M - 1; t >= 0; t--) {
      const double d = rhs(v, sv, sg, fac, t);
      y = fma(fac(0, t), y, d);
      v[t] = y;
    }
    ycarry = y;
    if constexpr (kUni) gcarry = lane_value(f[2][0], 0);
    double z = 0.0;
#pragma unroll
    for (int t = 0; t < M; t++) {
      z = fma(fac(2, t), z, fac(1, t) * v[t]);
      v[t] = z;
    }
    zin = v[0];
    store(v, sv, k);
    // resolved into the next chunk's carry below
    if (zlds) zouter[k][lane] = v[M - 1];
    else if (active && k + 1 < kend) zslot[(long)(k + 1) * kstr] = v[M - 1];
    if constexpr (!kUni) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  };

  double vA[M], sA[M], vB[M], sB[M];
  double svA[MS], svB[MS];
  double fA[NF][NQ], fB[NF][NQ];
  if (!bottom) {
    if (kend > kbeg) {
      issue(vA, svA, sA, fA, kbeg);
      for (int k = kbeg; k < kend; k += 2) {
        if (k + 1 < kend) issue(vB, svB, sB, fB, k + 1);
        process_down(vA, svA, sA, fA, k);
        if (k + 1 < kend) {
          if (k + 2 < kend) issue(vA, svA, sA, fA, k + 2);
          process_down(vB, svB, sB, fB, k + 1);
        }
      }
    }
  } else {
    if (kend > kbeg) {
      issue(vA, svA, sA, fA, kend - 1);
      for (int k = kend - 1; k >= kbeg; k -= 2) {
        if (k - 1 >= kbeg) issue(vB, svB, sB, fB, k - 1);
        process_up(vA, svA, sA, fA, k);
        if (k - 1 >= kbeg) {
          if (k - 2 >= kbeg) issue(vA, svA, sA, fA, k - 2);
          process_up(vB, svB, sB, fB, k - 1);
        }
      }
    }
  }
  // true value just past this wave's innermost chunk (0 at the line end)
  double xin = 0.0;
  if constexpr (TW) {
    zmid[wv][lane] = zin;
    __syncthreads();
    if (kmid < P) {
      const int mid = kmid * M;
      const double zt = zmid[0][lane], zb = zmid[1][lane];
      const double gt = Gf[(long)lc * n_pos + mid - 1];  // couples mid-1 to mid (top)
      const double gb = Gf[(long)lc * n_pos + mid];      // couples mid to mid-1 (bottom)
      const double xm1 = (zt + gt * zb) / (1.0 - gt * gb);
      xin = bottom ? xm1 : fma(gb, xm1, zb);
    }
  }
  // chunk carries, from the innermost chunk outwards:
  //   top:    sigma_k = zfirst_{k+1} + phi_{(k+1) start} sigma_{k+1}
  //   bottom: sigma_k = zlast_{k-1} + phi_{(k-1) end} sigma_{k-1}
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (active && kend > kbeg) {
    gdouble* so = zslot;
    const gdouble* ps = phiS + (long)line * P;
    double sigma = xin;
    constexpr int kB = 8;
    if (!bottom) {
      so[(long)(kend - 1) * kstr] = sigma;
      for (int k0 = kend - 2; k0 >= kbeg; k0 -= kB) {
        double ph[kB], zq[kB];
#pragma unroll
        for (int u = 0; u < kB; u++) {
          const int k = k0 - u;
          ph[u] = k >= kbeg ? ps[k + 1] : 0.0;
          zq[u] = k >= kbeg ? (zlds ? zouter[k + 1][lane] : so[(long)k * kstr]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kB; u++) {
          const int k = k0 - u;
          if (k >= kbeg) {
            sigma = fma(ph[u], sigma, zq[u]);
            so[(long)k * kstr] = sigma;
          }
        }
      }
    } else {
      so[(long)kbeg * kstr] = sigma;
      for (int k0 = kbeg + 1; k0 < kend; k0 += kB) {
        double ph[kB], zq[kB];
#pragma unroll
        for (int u = 0; u < kB; u++) {
          const int k = k0 + u;
          ph[u] = k < kend ? ps[k - 1] : 0.0;
          zq[u] = k < kend ? (zlds ? zouter[k - 1][lane] : so[(long)k * kstr]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kB; u++) {
          const int k = k0 + u;
          if (k < kend) {
            sigma = fma(ph[u], sigma, zq[u]);
            so[(long)k * kstr] = sigma;
          }
        }
      }
    }
  }
}

// Fine sweep of kGL consecutive lines per workgroup, one slice block of 64
// slices per line, two waves per line (the twisted form of k_fine_sweep, see
// there): 2 * kGL waves. The lines of a workgroup lie in one chunk of the
// previous sweep (M is a multiple of kGL and groups start at multiples of
// kGL), so their pending-correction carries sigma_prev[k][p][slice] are the
// same rows: each wave of a half loads M / kGL of the chunk's rows, stages
// them in LDS, and after a barrier every wave of the half reads the chunk's
// carries from there. That cuts the carry loads per wave by kGL, which leaves
// a wave's limited number of outstanding memory operations to the values
// themselves. The two halves run the same number of rounds (one chunk each
// per round, the shorter half idle in its last one) so that every wave
// reaches every barrier.
constexpr int kGL = 4;  // lines per workgroup of the grouped sweep

template <int M, int DIR, bool HP, bool FT, bool ZG>
__global__ __launch_bounds__(2 * kGL * kWave) void k_fine_sweep_g(
    const DimInst* __restrict__ insts, const WorkItem* __restrict__ work, int step) {
  constexpr int L = kWave;
  constexpr int NF = FT ? 4 + kMaxForcing : 4;
  constexpr int Q = M / kGL;  // carry rows staged by each wave per chunk
  constexpr int QO = (Q + 1) / 2;  // 16-byte loads for them: two rows per load
  static_assert(M % kGL == 0, "the chunk's carry rows are split over the group's waves");
  static_assert(!FT || DIR == 0, "the source enters the first (x) stage");
  constexpr int kMaxChunks = (kLineSeg + M - 1) / M;
  __shared__ __attribute__((aligned(16))) double ssig[HP ? 2 : 1][HP ? 2 : 1][HP ? M : 1][kWave];  // [half][buffer][row][slice]
  __shared__ double zouter[kGL][kMaxChunks][kWave];
  __shared__ double zmid[2][kGL][kWave];

  const WorkItem w = work[blockIdx.x];
  const DimInst& I = insts[w.inst];
  if (step >= I.steps) return;  // this instance has finished its fine steps
  if (I.active && !I.active[I.idx]) return;  // converged instance
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int half = wid / kGL;  // 0: top part of the line, 1: bottom part
  const int q = wid - half * kGL;  // line of the group
  const bool bottom = half == 1;

  const int n_lines = DIR == 0 ? I.ny : I.nx;
  const int n_pos = DIR == 0 ? I.nx : I.ny;
  const int P = DIR == 0 ? I.Px : I.Py;
  const int kmid = min(DIR == 0 ? I.twx : I.twy, P);
  const int kbeg = bottom ? kmid : 0, kend = bottom ? P : kmid;
  const int nmine = kend - kbeg;
  const int nrounds = max(kmid, P - kmid);
  const int nl_prev = n_pos;
  const long pstr = DIR == 0 ? (long)L : (long)I.nx * L;
  const long lstr = DIR == 0 ? (long)I.nx * L : (long)L;
  const gdv2* RG = (const gdv2*)gp(DIR == 0 ? I.fxRG : I.fyRG);
  const gdouble* Gf = gp(DIR == 0 ? I.fxG : I.fyG);
  const gdouble* phiS = gp(DIR == 0 ? I.fxPhiS : I.fyPhiS);
  const gdouble* phiPrev = gp(DIR == 0 ? I.fyPhiC : I.fxPhiC);
  const gdouble* sigPrev = DIR == 0 ? gp(I.sigY) + (long)w.b * I.Py * I.nx * L
                                    : gp(I.sigX) + (long)w.b * I.Px * I.ny * L;
  gdouble* sigOut = DIR == 0 ? gp(I.sigX) + (long)w.b * I.Px * I.ny * L
                             : gp(I.sigY) + (long)w.b * I.Py * I.nx * L;

  const int line0 = w.group * kGL;
  const int line = line0 + q;
  const bool active = line < n_lines;  // wave-uniform
  const int lc = active ? line : n_lines - 1;  // clamped for in-bounds loads
  // chunk outer values in LDS, or (ZG: launches with lines longer than the
  // LDS store holds) in the carry slots they resolve into (see k_fine_sweep)
  constexpr bool zlds = !ZG;
  gdouble* zslot = sigOut + (long)lc * L + lane;
  const long kstr = (long)n_lines * L;
  const gdouble* zrow_u = gp(I.Z) + w.b * I.slab + (long)lc * lstr;
  // carry rows of the group's chunk of the previous sweep
  const gdouble* sgrow_u = sigPrev + ((long)(line0 / M) * nl_prev) * L;
  const long frow = (long)lc * n_pos;
  const unsigned usl = (unsigned)lane;
  const long zo = I.zout;
  double gl[kMaxForcing] = {};
  const gdouble* fS = FT ? gp(I.fS) : nullptr;
  if constexpr (FT) {
    const int slice = w.b * L + lane;
    const long nst = (long)I.N * I.steps;
    const long gi = (long)(slice < I.N ? slice : 0) * I.steps + step;
#pragma unroll
    for (int m = 0; m < kMaxForcing; m++) {
      const double g = gp(I.fgf)[m * nst + gi];
      gl[m] = slice < I.N ? g : 0.0;
    }
  }
  // chunk processed by this wave in round r
  auto chunk_of = [&](int r) { return bottom ? P - 1 - r : r; };
  // carry staging: load o of this wave covers rows q Q + 2 o (lanes 0-31) and
  // q Q + 2 o + 1 (lanes 32-63) of the chunk, two slices per lane
  const int srow = lane >> 5, sslc = 2 * (lane & 31);
  auto issue = [&](double (&v)[M], dv2 (&sq)[QO], double (&f)[NF], int r) {
    const int k = chunk_of(r);
    const int p0 = k * M;
    const int cnt = min(M, n_pos - p0);
    // issue order: factors, carry rows, values. A wait for an older load is a wait
    // for everything issued before it, so the loads whose registers are freed (or
    // staged) first come first.
    const long idx = frow + p0 + (lane < cnt ? lane : 0);
    const dv2 rg = RG[idx];
    double fphi = 0.0;
    if constexpr (HP) fphi = phiPrev[idx];
    double fsrc[kMaxForcing] = {};
    if constexpr (FT) {
#pragma unroll
      for (int m = 0; m < kMaxForcing; m++) fsrc[m] = fS[m * I.npts + idx];
    }
    if constexpr (HP) {
      const gdouble* sc = sgrow_u + (long)p0 * L + sslc;
#pragma unroll
      for (int o = 0; o < QO; o++) {
        const int tr = q * Q + 2 * o + srow;
        const int tt = tr < cnt ? tr : 0;
        sq[o] = *(const gdv2*)(sc + (long)tt * L);
      }
    }
    const gdouble* zc = zrow_u + (long)p0 * pstr;
#pragma unroll
    for (int t = 0; t < M; t++) {
      const int tt = (cnt == M || t < cnt) ? t : 0;
      v[t] = (zc + (long)tt * pstr)[usl];
    }
    f[1] = rg.x;
    f[2] = rg.y;
    if constexpr (HP) f[3] = fphi;
    if constexpr (FT) {
#pragma unroll
      for (int m = 0; m < kMaxForcing; m++) f[4 + m] = fsrc[m];
    }
  };

  double ycarry = 0.0, gcarry = 0.0, zin = 0.0;
  auto round = [&](double (&v)[M], dv2 (&sq)[QO], double (&f)[NF], int r) {
    const bool mine = r < nmine;  // wave-uniform
    const int buf = r & 1;
    if constexpr (HP) {
      if (mine) {
#pragma unroll
        for (int o = 0; o < QO; o++) {
          const int row = 2 * o + srow;
          if (row < Q) *(dv2*)&ssig[half][buf][q * Q + row][sslc] = sq[o];
        }
      }
      __syncthreads();
    }
    if (!mine) return;
    const int k = chunk_of(r);
    const int p0 = k * M;
    const int cnt = min(M, n_pos - p0);
    auto rhs = [&](int t) -> double {
      double d = v[t];
      if constexpr (HP) d = fma(lane_value(f[3], t), ssig[half][buf][t][lane], d);
      if constexpr (FT) {
#pragma unroll
        for (int m = 0; m < kMaxForcing; m++) d = fma(gl[m], lane_value(f[4 + m], t), d);
      }
      return d;
    };
    double y = ycarry;
    if (!bottom) {
#pragma unroll
      for (int t = 0; t < M; t++) {
        const double e = t == 0 ? gcarry : lane_value(f[2], t - 1);
        y = fma(e, y, rhs(t));
        v[t] = y;
      }
      gcarry = lane_value(f[2], M - 1);
      double z = 0.0;
#pragma unroll
      for (int t = M - 1; t >= 0; t--) {
        z = fma(lane_value(f[2], t), z, lane_value(f[1], t) * v[t]);
        v[t] = z;
      }
      zin = v[M - 1];
      if (zlds) zouter[q][k][lane] = v[0];
      else if (active && k > kbeg) zslot[(long)(k - 1) * kstr] = v[0];
    } else {
#pragma unroll
      for (int t = M - 1; t >= 0; t--) {
        const double e = t == M - 1 ? gcarry : (t + 1 < cnt ? lane_value(f[2], t + 1) : 0.0);
        y = fma(e, y, rhs(t));
        v[t] = y;
      }
      gcarry = lane_value(f[2], 0);
      double z = 0.0;
#pragma unroll
      for (int t = 0; t < M; t++) {
        z = fma(lane_value(f[2], t), z, lane_value(f[1], t) * v[t]);
        v[t] = z;
      }
      zin = v[0];
      if (zlds) zouter[q][k][lane] = v[M - 1];
      else if (active && k + 1 < kend) zslot[(long)(k + 1) * kstr] = v[M - 1];
    }
    ycarry = y;
    if (active) {
      gdouble* zc = (gdouble*)zrow_u + (long)p0 * pstr;
      if (cnt == M) {
#pragma unroll
        for (int t = 0; t < M; t++) __builtin_nontemporal_store(v[t], &(zc + zo + (long)t * pstr)[usl]);
      } else {
#pragma unroll
        for (int t = 0; t < M; t++)
          if (t < cnt) __builtin_nontemporal_store(v[t], &(zc + zo + (long)t * pstr)[usl]);
      }
    }
  };

  double vA[M], vB[M], fA[NF], fB[NF];
  dv2 qA[QO], qB[QO];
  // the scheduling barriers keep each chunk's loads issued before the previous
  // chunk is processed (the compiler would otherwise sink them past the barrier
  // wait of the carry staging)
  if (nrounds > 0) {
    if (nmine > 0) issue(vA, qA, fA, 0);
    for (int r = 0; r < nrounds; r += 2) {
      if (r + 1 < nmine) issue(vB, qB, fB, r + 1);
      __builtin_amdgcn_sched_barrier(0);
      round(vA, qA, fA, r);
      __builtin_amdgcn_sched_barrier(0);
      if (r + 1 < nrounds) {
        if (r + 2 < nmine) issue(vA, qA, fA, r + 2);
        __builtin_amdgcn_sched_barrier(0);
        round(vB, qB, fB, r + 1);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  // interface of the two parts (see k_fine_sweep)
  zmid[half][q][lane] = zin;
  __syncthreads();
  double xin = 0.0;
  if (kmid < P) {
    const int mid = kmid * M;
    const double zt = zmid[0][q][lane], zb = zmid[1][q][lane];
    const double gt = Gf[frow + mid - 1];
    const double gb = Gf[frow + mid];
    const double xm1 = (zt + gt * zb) / (1.0 - gt * gb);
    xin = bottom ? xm1 : fma(gb, xm1, zb);
  }
  if (active && nmine > 0) {
    gdouble* so = zslot;
    const gdouble* ps = phiS + (long)line * P;
    double sigma = xin;
    constexpr int kB = 8;
    if (!bottom) {
      so[(long)(kend - 1) * kstr] = sigma;
      for (int k0 = kend - 2; k0 >= kbeg; k0 -= kB) {
        double ph[kB], zq[kB];
#pragma unroll
        for (int u = 0; u < kB; u++) {
          const int k = k0 - u;
          ph[u] = k >= kbeg ? ps[k + 1] : 0.0;
          zq[u] = k >= kbeg ? (zlds ? zouter[q][k + 1][lane] : so[(long)k * kstr]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kB; u++) {
          const int k = k0 - u;
          if (k >= kbeg) {
            sigma = fma(ph[u], sigma, zq[u]);
            so[(long)k * kstr] = sigma;
          }
        }
      }
    } else {
      so[(long)kbeg * kstr] = sigma;
      for (int k0 = kbeg + 1; k0 < kend; k0 += kB) {
        double ph[kB], zq[kB];
#pragma unroll
        for (int u = 0; u < kB; u++) {
          const int k = k0 + u;
          ph[u] = k < kend ? ps[k - 1] : 0.0;
          zq[u] = k < kend ? (zlds ? zouter[q][k - 1][lane] : so[(long)k * kstr]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kB; u++) {
          const int k = k0 + u;
          if (k < kend) {
            sigma = fma(ph[u], sigma, zq[u]);
            so[(long)k * kstr] = sigma;
          }
        }
      }
    }
  }
}

// -------------------------------------------------------- coarse sweeps ---
// One state (natural layout). Each line is solved exactly by one wave: lane l
// owns the K consecutive positions lK .. lK+K-1 of a segment of 64 K positions
// (the whole line when it has at most kLineSeg positions). The forward
// elimination y_p = e_p y_{p-1} + d_p and the back substitution
// x_p = g_p x_{p+1} + r_p y_p are affine recurrences: each lane composes its K
// maps, one inclusive scan of the 64 lane maps across the wave gives every lane
// its incoming value, and each lane re-runs its K steps from it. A line of one
// segment stays in registers between the two passes; a longer one is
// eliminated segment by segment downwards with the last y (and the last g, the
// next segment's first multiplier) carried across, the y of every segment but
// the last parked in the destination, and then substituted segment by segment
// upwards with the first x carried across.
//
// The factors are read in the lane-blocked layout [line][segment][c][lane]
// (position lane*K + c of the segment; one contiguous 512-byte segment per
// load). The state moves between its natural layout and the lanes through an
// LDS line buffer with one pad slot per 16 entries, which keeps both the
// position-ordered accesses of the global loads and stores and the lane-blocked
// accesses of the solve free of bank conflicts.

__device__ __forceinline__ int lds_pad(int q) { return q + (q >> 4); }

// doubles of one LDS line buffer for K positions per lane (odd: consecutive
// buffers start on different banks)
__host__ __device__ constexpr int line_buf_len(int K) { return 68 * K + 1; }

constexpr int kKMax = kLineSeg / kWave;  // positions per lane of a segment

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Every loop below runs all kKMax entries whatever K is: entries t >= K load
// from a clamped in-range address and are padded with identity maps (e = g = 1,
// r = 0, value 0), so there is no branch on K between a load and its use and the
// loads stay in flight together.

// Loads a segment's blocked factors (Rb, Gb at the segment) into registers.
__device__ __forceinline__ void load_line_factors(double (&gq)[kKMax], double (&rq)[kKMax], int K,
                                                  const gdouble* Rb, const gdouble* Gb,
                                                  int lane) {
#pragma unroll
  for (int t = 0; t < kKMax; t++) {
    const int tc = t < K ? t : 0;
    gq[t] = Gb[tc * kWave + lane];
    rq[t] = Rb[tc * kWave + lane];
  }
}

// Forward elimination y_p = e_p y_{p-1} + v_p, in place, of one lane-blocked
// segment (v zero past the line end and for t >= K; e_p = g_{p-1}, past the line
// end g = 0, so those positions stay 0). yin is y just before the segment and
// ein the multiplier of its first position (the g of the position before it),
// both 0 for a line's first segment; on return they hold the same two values
// for the next segment.
__device__ __forceinline__ void seg_forward(double (&v)[kKMax], int K, const double (&gq)[kKMax],
                                            double& yin, double& ein, int lane) {
  double glast = 0.0;
#pragma unroll
  for (int t = 0; t < kKMax; t++) glast = t == K - 1 ? gq[t] : glast;
  double e0 = __shfl_up(glast, 1, kWave);
  if (lane == 0) e0 = ein;
  double eq[kKMax];
#pragma unroll
  for (int t = 0; t < kKMax; t++) eq[t] = t < K ? (t == 0 ? e0 : gq[t - 1]) : 1.0;
  double A = 1.0, B = 0.0;
#pragma unroll
  for (int t = 0; t < kKMax; t++) {
    B = fma(eq[t], B, v[t]);
    A = eq[t] * A;
  }
  affine_scan_up(A, B, lane);
  const double ap = __shfl_up(A, 1, kWave), bp = __shfl_up(B, 1, kWave);
  double y = lane == 0 ? yin : fma(ap, yin, bp);  // y just before the lane's first position
#pragma unroll
  for (int t = 0; t < kKMax; t++) {
    y = fma(eq[t], y, v[t]);
    v[t] = y;
  }
  yin = lane_value(fma(A, yin, B), kWave - 1);
  ein = lane_value(glast, kWave - 1);
}

// Back substitution x_p = g_p x_{p+1} + r_p y_p, in place (v holds y), of one
// lane-blocked segment. xin is x just past the segment (0 for a line's last
// segment); on return it holds the segment's first x.
__device__ __forceinline__ void seg_backward(double (&v)[kKMax], int K, const double (&gq)[kKMax],
                                             const double (&rq)[kKMax], double& xin, int lane) {
  double gg[kKMax], rr[kKMax];
#pragma unroll
  for (int t = 0; t < kKMax; t++) {
    gg[t] = t < K ? gq[t] : 1.0;
    rr[t] = t < K ? rq[t] : 0.0;
  }
  double A = 1.0, B = 0.0;
#pragma unroll
  for (int t = kKMax - 1; t >= 0; t--) {
    B = fma(gg[t], B, rr[t] * v[t]);
    A = gg[t] * A;
  }
  affine_scan_down(A, B, lane);
  const double an = __shfl_down(A, 1, kWave), bn = __shfl_down(B, 1, kWave);
  double x = lane == kWave - 1 ? xin : fma(an, xin, bn);  // x just after the lane's last position
#pragma unroll
  for (int t = kKMax - 1; t >= 0; t--) {
    x = fma(gg[t], x, rr[t] * v[t]);
    v[t] = x;
  }
  xin = lane_value(fma(A, xin, B), 0);
}

// LDS line buffers hold one segment, so every buffer access below stays inside
// its own buffer for any K.
constexpr int kLineBuf = line_buf_len(kKMax);

// One row (contiguous, n values, S segments of 64 K): src -> dst (may alias);
// buf is the wave's LDS line buffer. With Sf != NULL the right-hand side also
// receives g0 S_0 + g1 S_1 (S_m at the row, S_1 = S_0 + spts).
template <bool SEG>
__device__ __forceinline__ void solve_row(const gdouble* src, gdouble* dst, const gdouble* Rb,
                                          const gdouble* Gb, int n, int K, int S_, double* buf,
                                          int lane, const gdouble* Sf = nullptr, long spts = 0,
                                          double g0 = 0.0, double g1 = 0.0) {
  const int S = SEG ? S_ : 1;  // one segment: a single pass (fewer live registers)
  const int SL = kWave * K;
  double v[kKMax], gq[kKMax], rq[kKMax];
  // v (position order) -> lane-blocked v, through the LDS buffer
  auto to_lanes = [&]() {
#pragma unroll
    for (int t = 0; t < kKMax; t++) buf[lds_pad(t * kWave + lane)] = v[t];
    wave_lds_fence();
#pragma unroll
    for (int t = 0; t < kKMax; t++) {
      const double x = buf[lds_pad(lane * K + (t < K ? t : 0))];
      v[t] = t < K ? x : 0.0;
    }
    wave_lds_fence();
  };
  // lane-blocked v -> dst[p0 + p], p < ns
  auto from_lanes = [&](int p0, int ns) {
#pragma unroll
    for (int t = 0; t < kKMax; t++)
      if (t < K) buf[lds_pad(lane * K + t)] = v[t];
    wave_lds_fence();
#pragma unroll
    for (int t = 0; t < kKMax; t++) {
      const int p = t * kWave + lane;
      if (p < ns) dst[p0 + p] = buf[lds_pad(p)];
    }
    wave_lds_fence();
  };
  auto load_seg = [&](const gdouble* a, int p0, int ns) {
#pragma unroll
    for (int t = 0; t < kKMax; t++) {
      const int p = t * kWave + lane;
      const double x = a[p0 + (p < ns ? p : 0)];
      v[t] = p < ns ? x : 0.0;  // p >= ns for every t >= K
    }
  };
  double yc = 0.0, ec = 0.0;
  for (int sg = 0; sg < S; sg++) {
    const int p0 = sg * SL, ns = min(n - p0, SL);
    load_seg(src, p0, ns);
    if (Sf) {  // wave-uniform
#pragma unroll
      for (int t = 0; t < kKMax; t++) {
        const int p = t * kWave + lane;
        const int pc = p0 + (p < ns ? p : 0);
        const double s0 = Sf[pc], s1 = Sf[spts + pc];
        v[t] = p < ns ? fma(g1, s1, fma(g0, s0, v[t])) : 0.0;
      }
    }
    load_line_factors(gq, rq, K, Rb + (long)sg * SL, Gb + (long)sg * SL, lane);
    to_lanes();
    seg_forward(v, K, gq, yc, ec, lane);
    if (sg + 1 < S) from_lanes(p0, ns);  // y parked in dst (read back by the same lanes)
  }
  double xc = 0.0;
  for (int sg = S - 1; sg >= 0; sg--) {
    const int p0 = sg * SL, ns = min(n - p0, SL);
    if (sg + 1 < S) {
      load_seg(dst, p0, ns);
      load_line_factors(gq, rq, K, Rb + (long)sg * SL, Gb + (long)sg * SL, lane);
      to_lanes();
    }
    seg_backward(v, K, gq, rq, xc, lane);
    from_lanes(p0, ns);
  }
}

constexpr int kRowsPerBlock = kCoarseRowsPerBlock;
constexpr int kColsPerBlock = kCoarseColsPerBlock;
constexpr int kColThreads = kWave * kColsPerBlock;
// staged elements per thread: a segment of the block's columns
constexpr int kStageIt = (kLineSeg * kColsPerBlock + kColThreads - 1) / kColThreads;

// Columns i0 .. i0 + kColsPerBlock - 1 of a state (S segments of 64 K rows),
// one column per wave, result into dst (mode 0), or combined with the parareal
// correction (mode 1: U_next = F + (g - G_old), G_old = g, increment) or the
// initial guess (mode 2: U_next = G_old = g). The columns are staged into one
// LDS line buffer each through row segments. Every global load of a segment
// (state, factors and the correction operands) is issued before its first LDS
// store. Columns of several segments park the y of all but the last segment in
// dst (which may alias src). Returns the thread's largest |change| bit pattern
// (mode 1).
template <bool SEG>
__device__ __forceinline__ unsigned long long solve_cols(
    const gdouble* src, int nx, int ny, int i0, int K, int S_, const gdouble* Rb, const gdouble* Gb,
    int mode, gdouble* dst, const gdouble* F, gdouble* Gold, gdouble* Unext, double* T,
    int tid) {
  const int S = SEG ? S_ : 1;  // one segment: a single pass (fewer live registers)
  const int lane = tid & (kWave - 1), wv = tid / kWave;
  const int col = i0 + wv;
  const int colc = col < nx ? col : nx - 1;  // clamped for the factor loads
  const int SL = kWave * K;
  const gdouble* Rl = Rb + (long)colc * SL * S;
  const gdouble* Gl = Gb + (long)colc * SL * S;
  double* buf = T + wv * kLineBuf;
  double st[kStageIt], gq[kKMax], rq[kKMax], v[kKMax];
  double fv[kStageIt], gv[kStageIt], uv[kStageIt];
  // rows [p0, p0 + ns) of the block's columns: thread entry u is row p0 + j,
  // column i0 + c with q = tid + u * kColThreads = j * kColsPerBlock + c
  auto stage_load = [&](const gdouble* a, int p0, int ns) {
#pragma unroll
    for (int u = 0; u < kStageIt; u++) {
      const int q = tid + u * kColThreads;
      const int j = q / kColsPerBlock, c = q - j * kColsPerBlock;
      const int i = i0 + c;
      const bool ok = q < ns * kColsPerBlock && i < nx;
      const double x = a[ok ? (long)(p0 + j) * nx + i : 0];
      st[u] = ok ? x : 0.0;
    }
  };
  auto corr_load = [&](int p0, int ns) {
    if (mode != 1) return;
#pragma unroll
    for (int u = 0; u < kStageIt; u++) {
      const int q = tid + u * kColThreads;
      const int j = q / kColsPerBlock, c = q - j * kColsPerBlock;
      const int i = i0 + c;
      const bool ok = q < ns * kColsPerBlock && i < nx;
      const long idx = ok ? (long)(p0 + j) * nx + i : 0;
      fv[u] = F[idx];
      gv[u] = Gold[idx];
      uv[u] = Unext[idx];
    }
  };
  auto stage_store = [&](int ns) {
#pragma unroll
    for (int u = 0; u < kStageIt; u++) {
      const int q = tid + u * kColThreads;
      const int j = q / kColsPerBlock, c = q - j * kColsPerBlock;
      if (q < ns * kColsPerBlock) T[c * kLineBuf + lds_pad(j)] = st[u];
    }
  };
  auto lanes_in = [&](int ns) {
#pragma unroll
    for (int t = 0; t < kKMax; t++) {
      const int p = lane * K + (t < K ? t : 0);
      const double x = buf[lds_pad(p)];
      v[t] = (t < K && p < ns) ? x : 0.0;
    }
  };
  auto lanes_out = [&]() {
#pragma unroll
    for (int t = 0; t < kKMax; t++)
      if (t < K) buf[lds_pad(lane * K + t)] = v[t];
  };
  double yc = 0.0, ec = 0.0;
  for (int sg = 0; sg < S; sg++) {
    const int p0 = sg * SL, ns = min(ny - p0, SL);
    stage_load(src, p0, ns);
    load_line_factors(gq, rq, K, Rl + (long)sg * SL, Gl + (long)sg * SL, lane);
    if (sg + 1 == S) corr_load(p0, ns);  // the last segment is the first to finish
    if (sg > 0) __syncthreads();  // the previous segment's LDS reads are done
    stage_store(ns);
    __syncthreads();
    if (col < nx) {  // wave-uniform
      lanes_in(ns);
      seg_forward(v, K, gq, yc, ec, lane);
      if (sg + 1 < S) lanes_out();
    }
    if (sg + 1 < S) {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kStageIt; u++) {
        const int q = tid + u * kColThreads;
        const int j = q / kColsPerBlock, c = q - j * kColsPerBlock;
        const int i = i0 + c;
        if (q < ns * kColsPerBlock && i < nx) dst[(long)(p0 + j) * nx + i] = T[c * kLineBuf + lds_pad(j)];
      }
    }
  }
  unsigned long long mx = 0;
  double xc = 0.0;
  for (int sg = S - 1; sg >= 0; sg--) {
    const int p0 = sg * SL, ns = min(ny - p0, SL);
    if (sg + 1 < S) {
      stage_load(dst, p0, ns);  // the parked y, read back by the threads that stored it
      load_line_factors(gq, rq, K, Rl + (long)sg * SL, Gl + (long)sg * SL, lane);
      corr_load(p0, ns);
      __syncthreads();  // the previous segment's output phase is done with T
      stage_store(ns);
      __syncthreads();
      if (col < nx) lanes_in(ns);
    }
    if (col < nx) {
      seg_backward(v, K, gq, rq, xc, lane);
      lanes_out();
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kStageIt; u++) {
      const int q = tid + u * kColThreads;
      const int j = q / kColsPerBlock, c = q - j * kColsPerBlock;
      const int i = i0 + c;
      if (q < ns * kColsPerBlock && i < nx) {
        const long idx = (long)(p0 + j) * nx + i;
        const double g = T[c * kLineBuf + lds_pad(j)];
        if (mode == 0) {
          dst[idx] = g;
        } else if (mode == 2) {
          Unext[idx] = g;
          Gold[idx] = g;
        } else {
          const double un = fv[u] + (g - gv[u]);
          const unsigned long long bits = abs_bits(un - uv[u]);
          mx = bits > mx ? bits : mx;
          Unext[idx] = un;
          Gold[idx] = g;
        }
      }
    }
  }
  return mx;
}

// Workgroups are dealt to the 8 XCDs round-robin by id; this maps launch slot
// `bid` of `nb` to a logical block so that each XCD holds a contiguous range
// (neighbouring column blocks share cache lines of the same rows).
__device__ __forceinline__ int xcd_block(int bid, int nb) {
  const int x = bid & 7, r = bid >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return x * per + min(x, rem) + r;
}

// x-lines (rows) of one state, one wave per row; with gtab the source
// sum_m gtab[m * gstride + gidx] S_m joins the right-hand side.
template <bool SEG>
__global__ __launch_bounds__(kWave* kRowsPerBlock) void k_coarse_x(
    const DimInst* __restrict__ insts, const double* __restrict__ src, double* __restrict__ dst,
    const double* __restrict__ Rb, const double* __restrict__ Gb, const double* __restrict__ gtab,
    long gidx, long gstride) {
  __shared__ double T[kRowsPerBlock * kLineBuf];
  const DimInst& I = insts[0];
  const int nx = I.nx, ny = I.ny, K = I.Kx, Sg = I.Sx;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int row = xcd_block(blockIdx.x, gridDim.x) * kRowsPerBlock + wv;
  if (row >= ny) return;  // whole wave; no block-level barrier follows
  const long base = (long)row * nx;
  const long fb = (long)row * kWave * K * Sg;
  const gdouble* S = gtab ? gp(I.fS) + base : nullptr;
  const double g0 = gtab ? gtab[gidx] : 0.0, g1 = gtab ? gtab[gstride + gidx] : 0.0;
  solve_row<SEG>(gp(src) + base, gp(dst) + base, gp(Rb) + fb, gp(Gb) + fb, nx, K, Sg,
                 T + wv * kLineBuf, lane, S, I.npts, g0, g1);
}

// y-lines (columns) of one state, kColsPerBlock columns per block: dst = result.
template <bool SEG>
__global__ __launch_bounds__(kColThreads) void k_coarse_y(const DimInst* __restrict__ insts,
                                                          const double* __restrict__ src,
                                                          double* __restrict__ dst,
                                                          const double* __restrict__ Rb,
                                                          const double* __restrict__ Gb) {
  __shared__ double T[kColsPerBlock * kLineBuf];
  const DimInst& I = insts[0];
  const int i0 = xcd_block(blockIdx.x, gridDim.x) * kColsPerBlock;
  solve_cols<SEG>(gp(src), I.nx, I.ny, i0, I.Ky, I.Sy, gp(Rb), gp(Gb), 0, gp(dst), nullptr,
                  nullptr, nullptr, T, threadIdx.x);
}

// ----------------------------------------------- batched coarse sweeps ---
// Same line solves, one launch per slice index n over the line blocks of every
// instance that has that slice (items ordered on the host per XCD).

template <bool SEG>
__global__ __launch_bounds__(kWave* kRowsPerBlock) void k_coarse_xb(
    const DimInst* __restrict__ insts, const LineItem* __restrict__ items, int n, int c,
    const double* __restrict__ U_base) {
  __shared__ double T[kRowsPerBlock * kLineBuf];
  const LineItem it = items[blockIdx.x];
  const DimInst& I = insts[it.inst];
  if (I.active && !I.active[I.idx]) return;
  if (n >= I.N || c >= I.cs) return;
  const int nx = I.nx, ny = I.ny, K = I.Kx, Sg = I.Sx;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int row = it.block * kRowsPerBlock + wv;
  if (row >= ny) return;  // whole wave
  const gdouble* src = c == 0 ? gp(U_base) + I.off_states + (long)n * I.npts : gp(I.tmp);
  const long base = (long)row * nx;
  // source at the end of coarse step c of slice n
  const gdouble* S = I.nforce ? gp(I.fS) + base : nullptr;
  const long nc = (long)I.N * I.cs, gi = (long)n * I.cs + c;
  const double g0 = I.nforce ? I.fgc[gi] : 0.0, g1 = I.nforce ? I.fgc[nc + gi] : 0.0;
  const long fb = (long)row * kWave * K * Sg;
  solve_row<SEG>(src + base, gp(I.tmp) + base, gp(I.cxRb) + fb, gp(I.cxGb) + fb, nx, K, Sg,
                 T + wv * kLineBuf, lane, S, I.npts, g0, g1);
}

// The increment of the correction (mode 1) goes to the instance's per-column-
// block partial maxima (plain read-modify-write: one block per entry per
// launch, launches in stream order); k_inc_reduce folds them afterwards.
template <bool SEG>
__global__ __launch_bounds__(kColThreads) void k_coarse_yb(
    const DimInst* __restrict__ insts, const LineItem* __restrict__ items, int n, int c, int mode,
    const double* __restrict__ F_base, double* __restrict__ G_base, double* __restrict__ U_base) {
  __shared__ double T[kColsPerBlock * kLineBuf];
  __shared__ unsigned long long wmax[kColsPerBlock];
  const LineItem it = items[blockIdx.x];
  const DimInst& I = insts[it.inst];
  if (I.active && !I.active[I.idx]) return;  // uniform over the block
  if (n >= I.N || c >= I.cs) return;
  const int tid = threadIdx.x;
  const int md = (c + 1 == I.cs) ? mode : 0;
  unsigned long long mx = solve_cols<SEG>(
      gp(I.tmp), I.nx, I.ny, it.block * kColsPerBlock, I.Ky, I.Sy, gp(I.cyRb), gp(I.cyGb), md,
      gp(I.tmp), gp(F_base) + I.off_slices + (long)n * I.npts,
      gp(G_base) + I.off_slices + (long)n * I.npts,
      gp(U_base) + I.off_states + (long)(n + 1) * I.npts, T, tid);
  if (md == 1) {
    mx = wave_max_u64(mx);
    if ((tid & (kWave - 1)) == 0) wmax[tid / kWave] = mx;
    __syncthreads();
    if (tid == 0) {
      unsigned long long m = wmax[0];
#pragma unroll
      for (int w = 1; w < kColsPerBlock; w++) m = wmax[w] > m ? wmax[w] : m;
      unsigned long long* slot = I.incp + it.block;
      if (m > *slot) *slot = m;
    }
  }
}

// inc[idx] = max(inc[idx], largest partial) for each instance with partials;
// one block per instance.
__global__ __launch_bounds__(256) void k_inc_reduce(const DimInst* __restrict__ insts,
                                                    unsigned long long* __restrict__ inc) {
  __shared__ unsigned long long wm[4];
  const DimInst& I = insts[blockIdx.x];
  if (!I.incp) return;  // block-uniform
  const int tid = threadIdx.x;
  const int nb = I.n_incp;
  unsigned long long m = 0;
  for (int b = tid; b < nb; b += 256) m = I.incp[b] > m ? I.incp[b] : m;
  m = wave_max_u64(m);
  if ((tid & (kWave - 1)) == 0) wm[tid / kWave] = m;
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 4; w++) m = wm[w] > m ? wm[w] : m;
    m = wm[0] > m ? wm[0] : m;
    if (m > inc[I.idx]) inc[I.idx] = m;
  }
}

// Lane-blocked copy of line-major factors: dst[l][s][c][lane] =
// src[l][s*64*K + lane*K + c] (0 past the line end), S segments per line. One
// thread per destination entry.
__global__ void k_block_factors(const double* __restrict__ src, int n_lines, int n_pos, int K,
                                int S, double* __restrict__ dst) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long seg = (long)kWave * K;
  const long per = seg * S;
  if (t >= (long)n_lines * per) return;
  const long l = t / per;
  const long r = t - l * per;
  const long sg = r / seg;
  const int rs = (int)(r - sg * seg);
  const int c = rs / kWave, lane = rs - c * kWave;
  const long p = sg * seg + (long)lane * K + c;
  dst[t] = p < n_pos ? src[l * n_pos + p] : 0.0;
}

__global__ void k_mask_update(const double* __restrict__ inc, int* __restrict__ active, int n,
                              double tol) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && active[i] && inc[i] < tol) active[i] = 0;
}

// ------------------------------------------------------ Douglas-Rachford ---
// S = dt A_y U (eq. DR_method needs the split operators applied to the step's
// input): (A_y U)_j = [a_{j+1}(U_{j+1} - U_j) - a_j(U_j - U_{j-1})]/h^2 - (c/2) U_j,
// U = 0 outside the grid. On the interleaved workspace the input values carry the
// pending correction of the previous y sweep, added here for all three rows.
__global__ void k_dr_stencil(const DimInst* __restrict__ insts, int has_prev, int step, int b_lo,
                             int b_hi) {
  const DimInst& I = insts[0];
  if (step >= I.steps) return;  // this instance has finished its fine steps
  if (I.active && !I.active[I.idx]) return;
  const int nx = I.nx, ny = I.ny, L = I.L, M = I.M, Py = I.Py;
  const long total = (long)(b_hi - b_lo) * I.slab;
  const long t0 = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t0 >= total) return;
  const long t = t0 + (long)b_lo * I.slab;
  const int l = (int)(t % L);
  const long node = t / L;
  const int b = (int)(node / ((long)nx * ny));
  const long rem = node - (long)b * nx * ny;
  const int j = (int)(rem / nx), i = (int)(rem - (long)j * nx);
  const gdouble* Zb = gp(I.Z) + b * I.slab;
  const gdouble* sig = gp(I.sigY) + (long)b * Py * nx * L;
  auto val = [&](int jj) -> double {
    if (jj < 0 || jj >= ny) return 0.0;
    double z = Zb[((long)jj * nx + i) * L + l];
    if (has_prev)
      z = fma(gp(I.fyPhiC)[(long)jj * nx + i], sig[((long)(jj / M) * nx + i) * L + l], z);
    return z;
  };
  const double um = val(j - 1), u0 = val(j), up = val(j + 1);
  const double aw = gp(I.ay)[(long)j * nx + i], ae = gp(I.ay)[(long)(j + 1) * nx + i];
  gp(I.drS)[t] = I.dr_coef * (ae * (up - u0) - aw * (u0 - um)) - I.dr_react * u0;
}

// Natural layout, one state: mode 0: S = dt A_y U, out = U + S; mode 1: out -= S.
__global__ void k_dr_stencil_nat(const DimInst* __restrict__ insts, const double* __restrict__ U,
                                 double* __restrict__ out, int mode) {
  const DimInst& I = insts[0];
  const int nx = I.nx, ny = I.ny;
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)nx * ny) return;
  gdouble* S = gp(I.drS);  // the first state's worth of the DR buffer
  if (mode == 1) {
    out[t] = out[t] - S[t];
    return;
  }
  const int j = (int)(t / nx), i = (int)(t - (long)j * nx);
  const double u0 = U[t];
  const double um = j > 0 ? U[t - nx] : 0.0, up = j + 1 < ny ? U[t + nx] : 0.0;
  const double aw = gp(I.ay)[(long)j * nx + i], ae = gp(I.ay)[(long)(j + 1) * nx + i];
  const double sv = I.dr_coef * (ae * (up - u0) - aw * (u0 - um)) - I.dr_react * u0;
  S[t] = sv;
  out[t] = u0 + sv;
}

// ---------------------------------------------------------------- source ---
// Z[b][node][l] += sum_m (dt g_m)(slice, step) S_m[node] for every node (DD
// fine workspace, where the first stage of a step touches every node).
__global__ void k_force_interleaved(const DimInst* __restrict__ insts, int step) {
  const DimInst& I = insts[0];
  const long total = (long)I.B * I.slab;
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int L = I.L;
  const int l = (int)(t % L);
  const long node_all = t / L;
  const int b = (int)(node_all / I.npts);
  const long node = node_all - (long)b * I.npts;
  const int slice = b * L + l;
  if (slice >= I.N) return;
  const long nst = (long)I.N * I.steps, gi = (long)slice * I.steps + step;
  double v = gp(I.Z)[t];
#pragma unroll
  for (int m = 0; m < kMaxForcing; m++) v = fma(gp(I.fgf)[m * nst + gi], gp(I.fS)[m * I.npts + node], v);
  gp(I.Z)[t] = v;
}

// u += sum_m gtab[m * gstride + gidx] S_m (one state).
__global__ void k_force_state(const DimInst* __restrict__ insts, double* __restrict__ u,
                              const double* __restrict__ gtab, long gidx, long gstride) {
  const DimInst& I = insts[0];
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= I.npts) return;
  double v = u[t];
#pragma unroll
  for (int m = 0; m < kMaxForcing; m++) v = fma(gtab[m * gstride + gidx], I.fS[m * I.npts + t], v);
  u[t] = v;
}

__global__ void k_fill_zero(double* __restrict__ p, size_t n) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.0;
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, size_t n) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) b[i] = a[i];
}

// ------------------------------------------------ partitioned fine sweeps ---

// One substep of the fine FIE step for the lines of direction DIR when a whole
// line of a slice block fits in one workgroup's registers (few slices), one
// workgroup per (instance, slice block, line). The line is cut into parts of Pl
// consecutive positions; a lane holds one (part, slice) pair, a wave 64 / nb
// parts of the block's nb slices, and each lane loads all of its part's values
// at once, so every load of the sweep is in flight together. With the line's
// plain LU (forward y_p = d_p + e_p y_{p-1}, e_p = g_{p-1}; back x_p = r_p y_p +
// g_p x_{p+1}; section 2.2, eq. FIE_method: each substep is an exact solve):
// started from y_{s-1} = 0, a part [s, e) gives y0, and the true y_p = y0_p +
// (e_s ... e_p) Yin with Yin the true y_{s-1}, so the parts' incoming values
// follow from a fold over the earlier parts of the maps Yin -> (e_s ... e_{e-1})
// Yin + y0_{e-1}. With the true y, the part's back substitution from x_e = 0
// gives x0_s, and x_s = x0_s + (g_s ... g_{e-1}) Xout with Xout = x_e the first
// value of the next part: a fold over the later parts gives each part's Xout,
// and a last back substitution from it gives the exact values. Every value is
// read and written once, and the output carries no pending correction.
template <int DIR, bool FT, int PL>
__global__ __launch_bounds__(kPartWaves* kWave, 4) void k_part_sweep(
    const DimInst* __restrict__ insts, const WorkItem* __restrict__ work, int step) {
  static_assert(!FT || DIR == 0, "the source enters the first (x) stage");
  __shared__ dv2 sRG[kLineSeg];  // (r_p, g_p) of the line
  __shared__ double sSrc[FT ? kMaxForcing : 1][FT ? kLineSeg : 1];
  // per lane: its scan within the wave (exchanged through LDS: the wave's lanes
  // run in lockstep, so each step's reads precede its writes without a
  // barrier); per wave and slice: the composed forward maps of its parts (A, B)
  // and the composed maps of their first values (C, D)
  __shared__ double sP[2][kPartWaves * kWave];
  __shared__ double sA[kPartWaves * kWave], sB[kPartWaves * kWave];
  __shared__ double sC[kPartWaves * kWave], sD[kPartWaves * kWave];

  const WorkItem w = work[blockIdx.x];
  const DimInst& I = insts[w.inst];
  if (step >= I.steps) return;  // this instance has finished its fine steps
  if (I.active && !I.active[I.idx]) return;  // converged instance
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid >> 6;
  const int L = I.Lp;                    // the partitioned sweeps' slice blocks
  const int nb = min(L, I.N - w.b * L);  // slices of this block
  const int G = kWave / nb;              // parts per wave
  const int gq = lane / nb, sl = lane - gq * nb;
  const int q = wv * G + gq;             // this lane's part
  const int n_pos = DIR == 0 ? I.nx : I.ny;
  const int Pl = DIR == 0 ? I.plx : I.ply;
  const int Pn = (n_pos + Pl - 1) / Pl;
  const bool act = gq < G && q < Pn;
  const int s0 = act ? q * Pl : 0;
  const int cnt = act ? min(Pl, n_pos - s0) : 0;
  const int line = w.group;
  const long pstr = DIR == 0 ? (long)L : (long)I.nx * L;
  const long lstr = DIR == 0 ? (long)I.nx * L : (long)L;
  const long base = w.b * I.slabp + (long)line * lstr + (long)s0 * pstr + (act ? sl : 0);
  const gdouble* zin = gp(I.Z) + base;
  gdouble* zst = gp(I.Z) + I.zout + base;

  // the part's values (positions past its end reload its first one)
  double v[PL];
#pragma unroll
  for (int t = 0; t < PL; t++) v[t] = t < Pl ? zin[(long)(t < cnt ? t : 0) * pstr] : 0.0;
  // the line's factors and source rows, staged for every lane (registers first,
  // so that one wait covers them)
  const gdv2* RG = (const gdv2*)(DIR == 0 ? I.pxRG : I.pyRG) + (long)line * n_pos;
  const int nthr = blockDim.x;
  const int nf = FT ? I.nforce : 0;  // source terms in use (the other rows are zero)
  constexpr int KS = 4;
  dv2 rg_st[KS];
  double src_st[FT ? KS : 1][FT ? kMaxForcing : 1];
#pragma unroll
  for (int k = 0; k < KS; k++) {
    const int p = tid + k * nthr;
    if (p < n_pos) {
      rg_st[k] = RG[p];
      if constexpr (FT) {
#pragma unroll
        for (int m = 0; m < kMaxForcing; m++)
          src_st[k][m] = m < nf ? gp(I.fS)[m * I.npts + (long)line * I.nx + p] : 0.0;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < KS; k++) {
    const int p = tid + k * nthr;
    if (p < n_pos) {
      sRG[p] = rg_st[k];
      if constexpr (FT) {
#pragma unroll
        for (int m = 0; m < kMaxForcing; m++) sSrc[m][p] = src_st[k][m];
      }
    }
  }
  for (int p = tid + KS * nthr; p < n_pos; p += nthr) {  // workgroups of fewer than 4 waves
    sRG[p] = RG[p];
    if constexpr (FT) {
#pragma unroll
      for (int m = 0; m < kMaxForcing; m++)
        sSrc[m][p] = m < nf ? gp(I.fS)[m * I.npts + (long)line * I.nx + p] : 0.0;
    }
  }
  // source: dt * g_m of this lane's slice at this step
  double gl[kMaxForcing] = {};
  if constexpr (FT) {
    const int slice = w.b * L + sl;
    const long nst = (long)I.N * I.steps;
#pragma unroll
    for (int m = 0; m < kMaxForcing; m++)
      gl[m] = (act && slice < I.N) ? gp(I.fgf)[m * nst + (long)slice * I.steps + step] : 0.0;
  }
  __syncthreads();

  // The recurrences run over all PL positions with clamped factor reads and
  // keep only the part's own steps (no branches, so the LDS reads can be issued
  // ahead); values past the part's end are never stored.
  const int last = n_pos - 1;
  // forward elimination of the part from y_{s-1} = 0
  double y = 0.0, psi = 1.0;
#pragma unroll
  for (int t = 0; t < PL; t++) {
    const int p = min(s0 + t, last);
    const bool ok = t < cnt;
    const double ep = sRG[p > 0 ? p - 1 : 0].y;
    const double e = p > 0 ? ep : 0.0;
    double d = v[t];
    if constexpr (FT) {
#pragma unroll
      for (int m = 0; m < kMaxForcing; m++) d = fma(gl[m], sSrc[m][p], d);
    }
    const double yn = fma(e, y, d);
    v[t] = yn;
    y = ok ? yn : y;
    psi = ok ? psi * e : psi;
  }
  // Yin of each part: the composition of the earlier parts' forward maps
  // y -> a y + b (a = psi at the part's end, b = y0 there) applied to 0; lanes
  // without a part carry the identity. An inclusive scan over this wave's parts
  // (lanes nb apart, same slice), each wave's total map through LDS folded over
  // the earlier waves, then the scan of the part before this one.
  const int nw = blockDim.x / kWave;
  {
    double fa = act ? psi : 1.0, fb = act ? y : 0.0;
    sP[0][tid] = fa;
    sP[1][tid] = fb;
#pragma unroll 1
    for (int k = 1; k < G; k <<= 1) {
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      const int src = gq >= k ? tid - k * nb : tid;
      const double pa = sP[0][src], pb = sP[1][src];
      if (gq >= k) {
        fb = fma(fa, pb, fb);
        fa *= pa;
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      sP[0][tid] = fa;
      sP[1][tid] = fb;
    }
    if (gq == G - 1) {
      sA[wv * kWave + sl] = fa;
      sB[wv * kWave + sl] = fb;
    }
  }
  __syncthreads();
  double Y = 0.0;
#pragma unroll 1
  for (int k = 0; k < wv; k++) Y = fma(sA[k * kWave + sl], Y, sB[k * kWave + sl]);
  if (gq >= 1) Y = fma(sP[0][tid - nb], Y, sP[1][tid - nb]);
  // true y of the part, and its back substitution from x_e = 0
  double dy = Y;
#pragma unroll
  for (int t = 0; t < PL; t++) {
    const int p = min(s0 + t, last);
    const double ep = sRG[p > 0 ? p - 1 : 0].y;
    dy *= p > 0 ? ep : 0.0;
    v[t] += dy;
  }
  double x = 0.0, phi = 1.0;
#pragma unroll
  for (int t = PL - 1; t >= 0; t--) {
    const bool ok = t < cnt;
    const dv2 rg = sRG[min(s0 + t, last)];
    const double xn = fma(rg.x, v[t], rg.y * x);
    x = ok ? xn : x;
    phi = ok ? phi * rg.y : phi;
  }
  // Xout of each part: its first value x_s = C Xout + D (C = the product of g
  // over the part, D = x0_s) composed over the later parts from the line end
  // (Xout = 0 after the last part), the same way in the other direction.
  __syncthreads();  // every lane has read its scan entries
  {
    double cc = act ? phi : 1.0, cd = act ? x : 0.0;
    sP[0][tid] = cc;
    sP[1][tid] = cd;
#pragma unroll 1
    for (int k = 1; k < G; k <<= 1) {
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      const int src = gq + k < G ? tid + k * nb : tid;
      const double na = sP[0][src], nd = sP[1][src];
      if (gq + k < G) {
        cd = fma(cc, nd, cd);
        cc *= na;
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      sP[0][tid] = cc;
      sP[1][tid] = cd;
    }
    if (gq == 0) {
      sC[wv * kWave + sl] = cc;
      sD[wv * kWave + sl] = cd;
    }
  }
  __syncthreads();
  double X = 0.0;
#pragma unroll 1
  for (int k = nw - 1; k > wv; k--) X = fma(sC[k * kWave + sl], X, sD[k * kWave + sl]);
  if (gq + 1 < G) X = fma(sP[0][tid + nb], X, sP[1][tid + nb]);
  x = X;
#pragma unroll
  for (int t = PL - 1; t >= 0; t--) {
    const bool ok = t < cnt;
    const dv2 rg = sRG[min(s0 + t, last)];
    const double xn = fma(rg.x, v[t], rg.y * x);
    x = ok ? xn : x;
    if (ok) zst[(long)t * pstr] = xn;
  }
}

}  // namespace

// ------------------------------------------------------------- launchers ---

hipError_t launch_faces_from_theta_2d(const double* theta, int nx, int ny, double* ax, double* ay,
                                      hipStream_t s) {
  long total = (long)ny * (nx + 1) + (long)(ny + 1) * nx;
  int blocks = (int)((total + 255) / 256);
  hipLaunchKernelGGL(k_faces_from_theta_2d, dim3(blocks), dim3(256), 0, s, theta, nx, ny, ax, ay);
  return hipGetLastError();
}

hipError_t launch_faces_from_theta_1d(const double* theta, int nx, double* ax, hipStream_t s) {
  int blocks = (nx + 1 + 255) / 256;
  hipLaunchKernelGGL(k_faces_from_theta_1d, dim3(blocks), dim3(256), 0, s, theta, nx, ax);
  return hipGetLastError();
}

hipError_t launch_factorize(const FactorJob& job, hipStream_t s) {
  int blocks = (job.n_lines + 63) / 64;
  hipLaunchKernelGGL(k_factorize, dim3(blocks), dim3(64), 0, s, job);
  return hipGetLastError();
}

hipError_t launch_factorize_twisted(const FactorJob& job, int mid, hipStream_t s) {
  hipLaunchKernelGGL(k_factorize_twisted, dim3((job.n_lines + 127) / 128), dim3(128), 0, s, job,
                     mid);
  return hipGetLastError();
}

hipError_t launch_interleave_pairs(const double* a, const double* b, long n, double* out,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_interleave_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n,
                     out);
  return hipGetLastError();
}

hipError_t launch_chunk_phi_twisted(const double* G, int n_lines, int n_pos, int M, int kmid,
                                    double* phiC, double* phiS, hipStream_t s) {
  hipLaunchKernelGGL(k_chunk_phi_twisted, dim3((n_lines + 127) / 128), dim3(128), 0, s, G, n_lines,
                     n_pos, M, kmid, phiC, phiS);
  return hipGetLastError();
}

hipError_t launch_chunk_phi(const double* G, int n_lines, int n_pos, int M, double* phiC,
                            double* phiS, hipStream_t s) {
  int blocks = (n_lines + 63) / 64;
  hipLaunchKernelGGL(k_chunk_phi, dim3(blocks), dim3(64), 0, s, G, n_lines, n_pos, M, phiC, phiS);
  return hipGetLastError();
}

hipError_t launch_to_interleaved(const DimInst* d_inst, const DimInst& h, const double* U_in,
                                 hipStream_t s, bool part) {
  if (part) {
    const long npts = (long)h.nx * h.ny;
    hipLaunchKernelGGL(k_to_part, dim3((unsigned)((npts + kPartTrNodes - 1) / kPartTrNodes), h.Bp),
                       dim3(256), 0, s, d_inst, U_in);
    return hipGetLastError();
  }
  dim3 grid((h.nx + 63) / 64, h.ny, h.B);
  hipLaunchKernelGGL(k_to_interleaved, grid, dim3(kTrThreads), 0, s, d_inst, U_in);
  return hipGetLastError();
}

hipError_t launch_from_interleaved(const DimInst* d_inst, const DimInst& h, double* F_out,
                                   bool with_corr, hipStream_t s, bool part) {
  if (part) {
    if (with_corr) return hipErrorInvalidValue;  // partitioned output is exact
    const long npts = (long)h.nx * h.ny;
    hipLaunchKernelGGL(k_from_part, dim3((unsigned)((npts + 255) / 256), h.Bp), dim3(256), 0, s,
                       d_inst, F_out);
    return hipGetLastError();
  }
  dim3 grid((h.nx + 63) / 64, h.ny, h.B);
  hipLaunchKernelGGL(k_from_interleaved, grid, dim3(kTrThreads), 0, s, d_inst, F_out,
                     (int)with_corr);
  return hipGetLastError();
}

template <int L, int M, int DIR, bool HP, int SGN, bool FT, bool TW>
static hipError_t launch_sweep_t(const DimInst* d_insts, const WorkItem* d_work, int n_work,
                                 int step, hipStream_t s) {
  hipLaunchKernelGGL((k_fine_sweep<L, M, DIR, HP, SGN, FT, TW>), dim3(n_work),
                     dim3(TW ? 2 * kWave : kWave), 0, s, d_insts, d_work, step);
  return hipGetLastError();
}

// x sweep: pending correction (hp), DR array added (SGN), source (FT)
template <int L, int M, int SGN, bool TW>
static hipError_t launch_sweep_x(const DimInst* d_insts, const WorkItem* d_work, int n_work,
                                 int has_prev, int step, hipStream_t s, bool forced) {
  if (forced)
    return has_prev ? launch_sweep_t<L, M, 0, true, SGN, true, TW>(d_insts, d_work, n_work, step, s)
                    : launch_sweep_t<L, M, 0, false, SGN, true, TW>(d_insts, d_work, n_work, step, s);
  return has_prev ? launch_sweep_t<L, M, 0, true, SGN, false, TW>(d_insts, d_work, n_work, step, s)
                  : launch_sweep_t<L, M, 0, false, SGN, false, TW>(d_insts, d_work, n_work, step, s);
}

template <int L, int M, bool TW>
static hipError_t launch_sweep_lm(const DimInst* d_insts, const WorkItem* d_work, int n_work,
                                  int dir, int has_prev, int step, hipStream_t s, int sgn,
                                  bool forced) {
  if (sgn != 0) {  // Douglas-Rachford (short chunks only): x adds S, y subtracts it
    if constexpr (M == kDRChunk) {
      if (dir == 0)
        return launch_sweep_x<L, M, 1, TW>(d_insts, d_work, n_work, has_prev, step, s, forced);
      return launch_sweep_t<L, M, 1, true, -1, false, TW>(d_insts, d_work, n_work, step, s);
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (dir == 0)
    return launch_sweep_x<L, M, 0, TW>(d_insts, d_work, n_work, has_prev, step, s, forced);
  return has_prev ? launch_sweep_t<L, M, 1, true, 0, false, TW>(d_insts, d_work, n_work, step, s)
                  : launch_sweep_t<L, M, 1, false, 0, false, TW>(d_insts, d_work, n_work, step, s);
}

template <int M, bool TW>
static hipError_t launch_sweep_m(const DimInst* d_insts, const WorkItem* d_work, int n_work, int L,
                                 int dir, int has_prev, int step, hipStream_t s, int sgn,
                                 bool f) {
  switch (L) {
    case 8: return launch_sweep_lm<8, M, TW>(d_insts, d_work, n_work, dir, has_prev, step, s, sgn, f);
    case 16: return launch_sweep_lm<16, M, TW>(d_insts, d_work, n_work, dir, has_prev, step, s, sgn, f);
    case 32: return launch_sweep_lm<32, M, TW>(d_insts, d_work, n_work, dir, has_prev, step, s, sgn, f);
    case 64: return launch_sweep_lm<64, M, TW>(d_insts, d_work, n_work, dir, has_prev, step, s, sgn, f);
    default: return hipErrorInvalidValue;
  }
}

template <bool TW>
static hipError_t launch_sweep_tw(const DimInst* d_insts, const WorkItem* d_work, int n_work,
                                  int L, int M, int dir, int has_prev, int step, hipStream_t s,
                                  int sgn, bool forced) {
  switch (M) {
    case 16:
      return launch_sweep_m<16, TW>(d_insts, d_work, n_work, L, dir, has_prev, step, s, sgn, forced);
    case 20:
      return launch_sweep_m<20, TW>(d_insts, d_work, n_work, L, dir, has_prev, step, s, sgn, forced);
    case 24:
      return launch_sweep_m<24, TW>(d_insts, d_work, n_work, L, dir, has_prev, step, s, sgn, forced);
    case 32:
      return launch_sweep_m<32, TW>(d_insts, d_work, n_work, L, dir, has_prev, step, s, sgn, forced);
    default: return hipErrorInvalidValue;
  }
}

template <int M, bool ZG>
static hipError_t launch_sweep_gz(const DimInst* d_insts, const WorkItem* d_work, int n_work,
                                  int dir, int has_prev, int step, hipStream_t s, bool forced) {
  const dim3 grid(n_work), block(2 * kGL * kWave);
  if (dir == 1) {
    if (has_prev)
      hipLaunchKernelGGL((k_fine_sweep_g<M, 1, true, false, ZG>), grid, block, 0, s, d_insts, d_work, step);
    else
      hipLaunchKernelGGL((k_fine_sweep_g<M, 1, false, false, ZG>), grid, block, 0, s, d_insts, d_work, step);
  } else if (forced) {
    if (has_prev)
      hipLaunchKernelGGL((k_fine_sweep_g<M, 0, true, true, ZG>), grid, block, 0, s, d_insts, d_work, step);
    else
      hipLaunchKernelGGL((k_fine_sweep_g<M, 0, false, true, ZG>), grid, block, 0, s, d_insts, d_work, step);
  } else {
    if (has_prev)
      hipLaunchKernelGGL((k_fine_sweep_g<M, 0, true, false, ZG>), grid, block, 0, s, d_insts, d_work, step);
    else
      hipLaunchKernelGGL((k_fine_sweep_g<M, 0, false, false, ZG>), grid, block, 0, s, d_insts, d_work, step);
  }
  return hipGetLastError();
}

template <int M>
static hipError_t launch_sweep_g(const DimInst* d_insts, const WorkItem* d_work, int n_work,
                                 int dir, int has_prev, int step, hipStream_t s, bool forced,
                                 bool long_lines) {
  return long_lines
             ? launch_sweep_gz<M, true>(d_insts, d_work, n_work, dir, has_prev, step, s, forced)
             : launch_sweep_gz<M, false>(d_insts, d_work, n_work, dir, has_prev, step, s, forced);
}

int lds_chunk_lines(int M) { return (kLineSeg + M - 1) / M; }

int grouped_lines() { return kGL; }

hipError_t launch_fine_sweep(const DimInst* d_insts, const WorkItem* d_work, int n_work, int L,
                             int M, int dir, int has_prev, int step, hipStream_t s, int sgn,
                             bool forced, bool twisted, bool grouped, bool long_lines) {
  if (forced && dir != 0) return hipErrorInvalidValue;
  if (grouped) {
    if (L != kWave || sgn != 0 || !twisted) return hipErrorInvalidValue;
    switch (M) {
      case 20: return launch_sweep_g<20>(d_insts, d_work, n_work, dir, has_prev, step, s, forced, long_lines);
      case 24: return launch_sweep_g<24>(d_insts, d_work, n_work, dir, has_prev, step, s, forced, long_lines);
      case 32: return launch_sweep_g<32>(d_insts, d_work, n_work, dir, has_prev, step, s, forced, long_lines);
      default: return hipErrorInvalidValue;
    }
  }
  return twisted ? launch_sweep_tw<true>(d_insts, d_work, n_work, L, M, dir, has_prev, step, s,
                                         sgn, forced)
                 : launch_sweep_tw<false>(d_insts, d_work, n_work, L, M, dir, has_prev, step, s,
                                          sgn, forced);
}

int part_positions(int n, int nb) {
  if (n < 1 || n > kLineSeg || nb < 1 || nb > kWave) return 0;
  const int parts = kPartWaves * (kWave / nb);
  const int Pl = (n + parts - 1) / parts;
  return Pl <= kPartMaxPL ? Pl : 0;
}

int part_waves(int n, int Pl, int nb) {
  const int Pn = (n + Pl - 1) / Pl, G = kWave / nb;
  return (Pn + G - 1) / G;
}

bool part_layout(int nx, int ny, int N, int* Lp, int* Bp, int* plx, int* ply) {
  for (int B = (N + kWave - 1) / kWave; B <= N; B++) {
    const int L = (N + B - 1) / B;
    if ((N + L - 1) / L != B) continue;  // the same blocks as fewer of them
    const int px = part_positions(nx, L), py = part_positions(ny, L);
    if (px > 0 && py > 0) {
      *Lp = L;
      *Bp = B;
      *plx = px;
      *ply = py;
      return true;
    }
  }
  return false;
}

template <int DIR, bool FT>
static hipError_t launch_part_t(const DimInst* d_insts, const WorkItem* d_work, int n_work,
                                int step, int waves, int pl, hipStream_t s) {
  const dim3 grid(n_work), block(waves * kWave);
  static_assert(kPartMaxPL == 24, "register arrays of 16 and 24 positions");
  if (pl <= 16)
    hipLaunchKernelGGL((k_part_sweep<DIR, FT, 16>), grid, block, 0, s, d_insts, d_work, step);
  else
    hipLaunchKernelGGL((k_part_sweep<DIR, FT, 24>), grid, block, 0, s, d_insts, d_work, step);
  return hipGetLastError();
}

hipError_t launch_part_sweep(const DimInst* d_insts, const WorkItem* d_work, int n_work, int dir,
                             int step, int waves, int pl, bool forced, hipStream_t s) {
  if ((forced && dir != 0) || waves < 1 || waves > kPartWaves || pl < 1 || pl > kPartMaxPL)
    return hipErrorInvalidValue;
  if (n_work == 0) return hipSuccess;
  if (dir == 0)
    return forced ? launch_part_t<0, true>(d_insts, d_work, n_work, step, waves, pl, s)
                  : launch_part_t<0, false>(d_insts, d_work, n_work, step, waves, pl, s);
  return launch_part_t<1, false>(d_insts, d_work, n_work, step, waves, pl, s);
}

int positions_per_lane(int n) {
  int p = 1;
  while (p * kWave < n && p * kWave < kLineSeg) p <<= 1;
  return p;
}

int line_segments(int n) {
  const int seg = kWave * positions_per_lane(n);
  return (n + seg - 1) / seg;
}

hipError_t launch_block_factors(const double* src, int n_lines, int n_pos, double* dst,
                                hipStream_t s) {
  const int K = positions_per_lane(n_pos), S = line_segments(n_pos);
  const long total = (long)n_lines * kWave * K * S;
  hipLaunchKernelGGL(k_block_factors, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src,
                     n_lines, n_pos, K, S, dst);
  return hipGetLastError();
}

hipError_t launch_coarse_x(const DimInst* d_inst, const DimInst& h, const double* src, double* dst,
                           bool fine, hipStream_t s, const double* gtab, long gidx, long gstride) {
  const dim3 grid((h.ny + kRowsPerBlock - 1) / kRowsPerBlock), block(kWave * kRowsPerBlock);
  if (h.Sx > 1)
    hipLaunchKernelGGL(k_coarse_x<true>, grid, block, 0, s, d_inst, src, dst,
                       fine ? h.fxRb : h.cxRb, fine ? h.fxGb : h.cxGb, gtab, gidx, gstride);
  else
    hipLaunchKernelGGL(k_coarse_x<false>, grid, block, 0, s, d_inst, src, dst,
                       fine ? h.fxRb : h.cxRb, fine ? h.fxGb : h.cxGb, gtab, gidx, gstride);
  return hipGetLastError();
}

hipError_t launch_coarse_y(const DimInst* d_inst, const DimInst& h, const double* src, double* dst,
                           bool fine, hipStream_t s) {
  const dim3 grid((h.nx + kColsPerBlock - 1) / kColsPerBlock), block(kColThreads);
  if (h.Sy > 1)
    hipLaunchKernelGGL(k_coarse_y<true>, grid, block, 0, s, d_inst, src, dst,
                       fine ? h.fyRb : h.cyRb, fine ? h.fyGb : h.cyGb);
  else
    hipLaunchKernelGGL(k_coarse_y<false>, grid, block, 0, s, d_inst, src, dst,
                       fine ? h.fyRb : h.cyRb, fine ? h.fyGb : h.cyGb);
  return hipGetLastError();
}

hipError_t launch_force_interleaved(const DimInst* d_inst, const DimInst& h, int step,
                                    hipStream_t s) {
  const long total = (long)h.B * h.slab;
  hipLaunchKernelGGL(k_force_interleaved, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     d_inst, step);
  return hipGetLastError();
}

hipError_t launch_force_state(const DimInst* d_inst, const DimInst& h, double* u,
                              const double* gtab, long gidx, long gstride, hipStream_t s) {
  hipLaunchKernelGGL(k_force_state, dim3((unsigned)((h.npts + 255) / 256)), dim3(256), 0, s,
                     d_inst, u, gtab, gidx, gstride);
  return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_coarse_xb(const DimInst* d_insts, const LineItem* items, int n_items, int n,
                            int c, const double* U_base, hipStream_t s, bool seg) {
  if (n_items <= 0) return hipSuccess;
  if (seg)
    hipLaunchKernelGGL(k_coarse_xb<true>, dim3(n_items), dim3(kWave * kRowsPerBlock), 0, s,
                       d_insts, items, n, c, U_base);
  else
    hipLaunchKernelGGL(k_coarse_xb<false>, dim3(n_items), dim3(kWave * kRowsPerBlock), 0, s,
                       d_insts, items, n, c, U_base);
  return hipGetLastError();
}

hipError_t launch_coarse_yb(const DimInst* d_insts, const LineItem* items, int n_items, int n,
                            int c, int mode, const double* F_base, double* G_base, double* U_base,
                            hipStream_t s, bool seg) {
  if (n_items <= 0) return hipSuccess;
  if (seg)
    hipLaunchKernelGGL(k_coarse_yb<true>, dim3(n_items), dim3(kColThreads), 0, s, d_insts, items,
                       n, c, mode, F_base, G_base, U_base);
  else
    hipLaunchKernelGGL(k_coarse_yb<false>, dim3(n_items), dim3(kColThreads), 0, s, d_insts, items,
                       n, c, mode, F_base, G_base, U_base);
  return hipGetLastError();
}

hipError_t launch_inc_reduce(const DimInst* d_insts, int n_inst, unsigned long long* inc,
                             hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_inc_reduce, dim3(n_inst), dim3(256), 0, s, d_insts, inc);
  return hipGetLastError();
}

hipError_t launch_dr_stencil(const DimInst* d_inst, const DimInst& h, int has_prev, int step,
                             int b_lo, int b_hi, hipStream_t s) {
  b_lo = std::max(0, b_lo);
  b_hi = std::min(h.B, b_hi);
  if (b_hi <= b_lo) return hipSuccess;
  const long total = (long)(b_hi - b_lo) * h.slab;
  hipLaunchKernelGGL(k_dr_stencil, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, d_inst,
                     has_prev, step, b_lo, b_hi);
  return hipGetLastError();
}

hipError_t launch_dr_stencil_nat(const DimInst* d_inst, const DimInst& h, const double* U,
                                 double* out, int mode, hipStream_t s) {
  const long total = (long)h.nx * h.ny;
  hipLaunchKernelGGL(k_dr_stencil_nat, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     d_inst, U, out, mode);
  return hipGetLastError();
}

hipError_t launch_mask_update(const double* inc, int* active, int n, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_mask_update, dim3((n + 255) / 256), dim3(256), 0, s, inc, active, n, tol);
  return hipGetLastError();
}

}  // namespace prk
