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
    job.E[idx] = e;
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

// ------------------------------------------------- interleave transposes ---

// Natural U[slice][j][i] -> Z[b][j][i][l]; one block per (64-column tile, row, block).
__global__ __launch_bounds__(kWave) void k_to_interleaved(const DimInst* __restrict__ insts,
                                                          const double* __restrict__ U) {
  __shared__ double tile[64][65];
  const DimInst& I = insts[0];
  if (I.active && !I.active[I.idx]) return;
  const int lane = threadIdx.x;
  const int i0 = blockIdx.x * 64, j = blockIdx.y, b = blockIdx.z;
  const int L = I.L, nx = I.nx;
  const long npts = (long)nx * I.ny;
  for (int s = 0; s < L; s++) {
    int slice = b * L + s;
    int i = i0 + lane;
    tile[s][lane] = (slice < I.N && i < nx) ? U[slice * npts + (long)j * nx + i] : 0.0;
  }
  __syncthreads();
  gdouble* Zb = gp(I.Z) + b * I.slab + ((long)j * nx + i0) * L;
  const int cnt = min(64, nx - i0);
  for (int q = lane; q < cnt * L; q += kWave) {
    int t = q / L, s = q - t * L;
    Zb[q] = tile[s][t];
  }
}

// Z (+ the pending chunk correction of the last y sweep) -> natural F[slice][j][i].
__global__ __launch_bounds__(kWave) void k_from_interleaved(const DimInst* __restrict__ insts,
                                                            double* __restrict__ F, int with_corr) {
  __shared__ double tile[64][65];
  const DimInst& I = insts[0];
  if (I.active && !I.active[I.idx]) return;
  const int lane = threadIdx.x;
  const int i0 = blockIdx.x * 64, j = blockIdx.y, b = blockIdx.z;
  const int L = I.L, nx = I.nx, M = I.M, Py = I.Py;
  const long npts = (long)nx * I.ny;
  const gdouble* Zb = gp(I.Z) + b * I.slab + ((long)j * nx + i0) * L;
  const int kj = j / M;
  const gdouble* sig = gp(I.sigY) + ((long)b * Py + kj) * nx * L;
  const gdouble* phiC = gp(I.fyPhiC) + (long)j * nx;
  const int cnt = min(64, nx - i0);
  for (int q = lane; q < cnt * L; q += kWave) {
    int t = q / L, s = q - t * L;
    int i = i0 + t;
    tile[s][t] = with_corr ? fma(phiC[i], sig[(long)i * L + s], Zb[q]) : Zb[q];
  }
  __syncthreads();
  for (int s = 0; s < L; s++) {
    int slice = b * L + s;
    if (slice < I.N && lane < cnt) F[slice * npts + (long)j * nx + i0 + lane] = tile[s][lane];
  }
}

// -------------------------------------------------------- fine sweeps ---

// One substep of the fine FIE step for every line of direction DIR of every
// slice of the work items' instances. Lanes = (line in group, slice); each
// wave walks its lines in chunks of M positions, holding one chunk in
// registers while the next one is being loaded. With HP, the pending chunk
// correction of the previous (other-direction) sweep is added on load.
// A partial last chunk is computed in full on clamped loads: the line's last
// back-substitution factor is 0, so the padded positions cannot leak into the
// real ones, and only real positions are stored.
template <int L, int M, int DIR, bool HP, int SGN = 0>
__global__ __launch_bounds__(kWave) void k_fine_sweep(const DimInst* __restrict__ insts,
                                                      const WorkItem* __restrict__ work,
                                                      int step) {
  constexpr int G = kWave / L;  // lines per wave
  constexpr bool kUni = (L == kWave);
  constexpr int NQ = kUni ? 1 : (G * M + kWave - 1) / kWave;
  static_assert(M <= kWave, "chunk longer than a wave");
  // factor staging when a wave holds several lines: [4][G][M+1]
  __shared__ double sF[kUni ? 1 : 4][kUni ? 1 : G][M + 1];
  // first value of every chunk of the wave's lines, resolved into carries at the end
  constexpr int kMaxChunks = (kMaxCoarseLine + M - 1) / M;
  __shared__ double zfirst[kMaxChunks][kWave];

  const WorkItem w = work[blockIdx.x];
  const DimInst& I = insts[w.inst];
  if (step >= I.steps) return;  // this instance has finished its fine steps
  if (I.active && !I.active[I.idx]) return;  // converged instance
  const int lane = threadIdx.x;
  const int gsub = lane / L;
  const int sl = lane - gsub * L;

  const int n_lines = DIR == 0 ? I.ny : I.nx;
  const int n_pos = DIR == 0 ? I.nx : I.ny;
  const int P = DIR == 0 ? I.Px : I.Py;
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
  // row of the previous sweep's carries for the chunk that holds this line
  const gdouble* sgRow = sigPrev + ((long)(lc / M) * nl_prev) * L + sl;
  gdouble* zbase = gp(I.Z) + w.b * I.slab + (long)lc * lstr + sl;
  const long frow = (long)line0 * n_pos;  // line-uniform factor row when kUni

  // With one line per wave the row pointers are wave-uniform: keep them apart
  // from the per-lane slice offset so addresses are scalar base + lane offset.
  const gdouble* zrow_u = gp(I.Z) + w.b * I.slab + (long)line0 * lstr;
  const gdouble* sgrow_u = sigPrev + ((long)(line0 / M) * nl_prev) * L;
  const unsigned usl = (unsigned)sl;  // lane offset (unsigned: scalar-base addressing)
  // DR: the stencil array lives at the same offsets as Z
  const long drOff = SGN != 0 ? (long)(I.drS - I.Z) : 0;
  auto issue = [&](double (&v)[M], double (&sg)[M], double (&f)[4][NQ], int k) {
    const int p0 = k * M;
    const int cnt = min(M, n_pos - p0);
    if constexpr (kUni) {
      const gdouble* zc = zrow_u + (long)p0 * pstr;
      const gdouble* sc = sgrow_u + (long)p0 * L;
#pragma unroll
      for (int t = 0; t < M; t++) {
        const int tt = (cnt == M || t < cnt) ? t : 0;
        v[t] = (zc + (long)tt * pstr)[usl];
        if constexpr (SGN != 0) v[t] = fma((double)SGN, (zc + drOff + (long)tt * pstr)[usl], v[t]);
        if constexpr (HP) sg[t] = (sc + (long)tt * L)[usl];
      }
    } else {
      const gdouble* zc = zbase + (long)p0 * pstr;
      const gdouble* sc = sgRow + (long)p0 * L;
      if (cnt == M) {
#pragma unroll
        for (int t = 0; t < M; t++) {
          v[t] = zc[t * pstr];
          if constexpr (SGN != 0) v[t] = fma((double)SGN, zc[drOff + t * pstr], v[t]);
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
          if constexpr (SGN != 0) v[t] = fma((double)SGN, zc[drOff + tt * pstr], v[t]);
          if constexpr (HP) sg[t] = sc[tt * L];
        }
      }
    }
    if constexpr (kUni) {
      const long idx = frow + p0 + (lane < cnt ? lane : 0);
      f[1][0] = R[idx];
      f[2][0] = Gf[idx];
      if constexpr (HP) f[3][0] = phiPrev[idx];
    } else {
#pragma unroll
      for (int qq = 0; qq < NQ; qq++) {
        const int q = lane + qq * kWave;
        const int g = q / M, t = q - g * M;
        const int ln = line0 + g, p = p0 + t;
        const bool ok = q < G * M && ln < n_lines && p < n_pos;
        const long idx = ok ? (long)ln * n_pos + p : 0;
        f[0][qq] = (ok && p > 0) ? Gf[idx - 1] : 0.0;  // e_p = g_{p-1}
        f[1][qq] = R[idx];
        f[2][qq] = Gf[idx];
        if constexpr (HP) f[3][qq] = phiPrev[idx];
      }
    }
  };

  double ycarry = 0.0;
  double gcarry = 0.0;  // g at the last position of the previous chunk (kUni path)
  auto process = [&](double (&v)[M], double (&sg)[M], double (&f)[4][NQ], int k) {
    const int p0 = k * M;
    const int cnt = min(M, n_pos - p0);
    if constexpr (!kUni) {
#pragma unroll
      for (int qq = 0; qq < NQ; qq++) {
        const int q = lane + qq * kWave;
        if (q < G * M) {
          const int g = q / M, t = q - g * M;
#pragma unroll
          for (int c = 0; c < (HP ? 4 : 3); c++) sF[c][g][t] = f[c][qq];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    auto fac = [&](int c, int t) -> double {
      if constexpr (kUni) {
        if (c == 0)  // e_p = g_{p-1}: the previous lane's g, or the last g of the previous chunk
          return t == 0 ? gcarry : lane_value(f[2][0], t - 1);
        return lane_value(f[c][0], t);
      } else {
        return sF[c][gsub][t];
      }
    };
    double y = ycarry;
#pragma unroll
    for (int t = 0; t < M; t++) {
      double d = v[t];
      if constexpr (HP) d = fma(fac(3, t), sg[t], d);
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
    if constexpr (kUni) {
      gdouble* zc = (gdouble*)zrow_u + (long)p0 * pstr;
      if (cnt == M) {
#pragma unroll
        for (int t = 0; t < M; t++) (zc + (long)t * pstr)[usl] = v[t];
      } else {
#pragma unroll
        for (int t = 0; t < M; t++)
          if (t < cnt) (zc + (long)t * pstr)[usl] = v[t];
      }
    } else if (active) {
      gdouble* zc = zbase + (long)p0 * pstr;
      if (cnt == M) {
#pragma unroll
        for (int t = 0; t < M; t++) zc[t * pstr] = v[t];
      } else {
#pragma unroll
        for (int t = 0; t < M; t++)
          if (t < cnt) zc[t * pstr] = v[t];
      }
    }
    zfirst[k][lane] = v[0];  // resolved into the chunk's carry below
    if constexpr (!kUni) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  };

  double vA[M], sA[M], vB[M], sB[M];
  double fA[4][NQ], fB[4][NQ];
  issue(vA, sA, fA, 0);
  for (int k = 0; k < P; k += 2) {
    if (k + 1 < P) issue(vB, sB, fB, k + 1);
    process(vA, sA, fA, k);
    if (k + 1 < P) {
      if (k + 2 < P) issue(vA, sA, fA, k + 2);
      process(vB, sB, fB, k + 1);
    }
  }
  // chunk carries: sigma_{P-1} = 0, sigma_k = zfirst_{k+1} + phi_{(k+1) start} sigma_{k+1}
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (active) {
    gdouble* so = sigOut + (long)line * L + sl;
    const long kstr = (long)n_lines * L;
    const gdouble* ps = phiS + (long)line * P;
    double sigma = 0.0;
    so[(long)(P - 1) * kstr] = 0.0;
    constexpr int kB = 8;
    for (int k0 = P - 2; k0 >= 0; k0 -= kB) {
      double ph[kB];
#pragma unroll
      for (int u = 0; u < kB; u++) {
        const int k = k0 - u;
        ph[u] = k >= 0 ? ps[k + 1] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kB; u++) {
        const int k = k0 - u;
        if (k >= 0) {
          sigma = fma(ph[u], sigma, zfirst[k + 1][lane]);
          so[(long)k * kstr] = sigma;
        }
      }
    }
  }
}

// -------------------------------------------------------- coarse sweeps ---
// One state (natural layout). Each line is solved exactly by one wave: lane l
// owns the K consecutive positions lK .. lK+K-1 (K*64 >= line length). The
// forward elimination y_p = e_p y_{p-1} + d_p and the back substitution
// x_p = g_p x_{p+1} + r_p y_p are affine recurrences: each lane composes its K
// maps, one inclusive scan of the 64 lane maps across the wave gives every lane
// its incoming value, and each lane re-runs its K steps from it. The line stays
// in registers between the two passes.

// positions per lane: the smallest power of two with 64 K >= n
__device__ __forceinline__ int chunks_pow2_dev(int n) {
  const int c = (n + kWave - 1) / kWave;
  int p = 1;
  while (p < c) p <<= 1;
  return p;
}

template <int KMAX>
__device__ __forceinline__ void line_solve_blocked(double (&v)[KMAX], int K, const gdouble* R,
                                                   const gdouble* Gf, int n, int lane) {
  const int p0 = lane * K;
  double gq[KMAX], rq[KMAX], eq[KMAX];
#pragma unroll
  for (int t = 0; t < KMAX; t++) {
    if (t < K) {
      const int p = p0 + t;
      const bool ok = p < n;
      gq[t] = ok ? Gf[p] : 0.0;
      rq[t] = ok ? R[p] : 0.0;
      eq[t] = ok ? (p > 0 ? Gf[p - 1] : 0.0) : 1.0;  // e_p = g_{p-1}; identity past the end
      if (!ok) v[t] = 0.0;
    }
  }
  // forward elimination
  double A = 1.0, B = 0.0;
#pragma unroll
  for (int t = 0; t < KMAX; t++)
    if (t < K) {
      B = fma(eq[t], B, v[t]);
      A = eq[t] * A;
    }
  affine_scan_up(A, B, lane);
  double y = __shfl_up(B, 1, kWave);  // value just before the lane's first position
  if (lane == 0) y = 0.0;
#pragma unroll
  for (int t = 0; t < KMAX; t++)
    if (t < K) {
      y = fma(eq[t], y, v[t]);
      v[t] = y;
    }
  // back substitution
  A = 1.0;
  B = 0.0;
#pragma unroll
  for (int t = KMAX - 1; t >= 0; t--)
    if (t < K) {
      B = fma(gq[t], B, rq[t] * v[t]);
      A = gq[t] * A;
    }
  affine_scan_down(A, B, lane);
  double x = __shfl_down(B, 1, kWave);  // value just after the lane's last position
  if (lane == kWave - 1) x = 0.0;
#pragma unroll
  for (int t = KMAX - 1; t >= 0; t--)
    if (t < K) {
      x = fma(gq[t], x, rq[t] * v[t]);
      v[t] = x;
    }
}

constexpr int kRowsPerBlock = kCoarseRowsPerBlock;

// x-lines (rows), one wave per row: coalesced along the row.
template <int NC>
__global__ __launch_bounds__(kWave* kRowsPerBlock) void k_coarse_x(
    const DimInst* __restrict__ insts, const double* __restrict__ src, double* __restrict__ dst,
    const double* __restrict__ FE, const double* __restrict__ FR, const double* __restrict__ FG) {
  const DimInst& I = insts[0];
  const int nx = I.nx, ny = I.ny;
  const int lane = threadIdx.x & (kWave - 1);
  const int row = blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6);
  if (row >= ny) return;  // whole wave
  const long base = (long)row * nx;
  double v[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) {
    int p = lane * NC + c;
    v[c] = p < nx ? src[base + p] : 0.0;
  }
  line_solve_blocked<NC>(v, NC, gp(FR) + base, gp(FG) + base, nx, lane);
#pragma unroll
  for (int c = 0; c < NC; c++) {
    int p = lane * NC + c;
    if (p < nx) dst[base + p] = v[c];
  }
}

constexpr int kColsPerBlock = kCoarseColsPerBlock;
constexpr int kTS = kColsPerBlock + 1;  // padded LDS row stride
// staged elements per thread: a column block of the longest line
constexpr int kStageIt = (kMaxCoarseLine * kColsPerBlock + kWave * kColsPerBlock - 1) /
                         (kWave * kColsPerBlock);

// y-lines (columns): a block of 16 columns is staged in LDS through
// 128-byte row segments, each wave solves one column, and the result is
// written back (mode 0), or combined with the parareal correction (mode 1:
// U_next = F + (g - G_old), G_old = g, increment) or the initial guess
// (mode 2: U_next = G_old = g).
template <int NC>
__global__ __launch_bounds__(kWave* kColsPerBlock) void k_coarse_y(
    const DimInst* __restrict__ insts, const double* __restrict__ src, double* __restrict__ dst,
    int mode, const double* __restrict__ F, double* __restrict__ Gold,
    double* __restrict__ Unext, unsigned long long* __restrict__ inc_bits,
    const double* __restrict__ FE, const double* __restrict__ FR, const double* __restrict__ FG) {
  extern __shared__ double T[];  // [ny][kTS]
  const DimInst& I = insts[0];
  const int nx = I.nx, ny = I.ny;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wv = tid >> 6;
  const int i0 = blockIdx.x * kColsPerBlock;
  const int total = ny * kColsPerBlock;
  {
    double st[kStageIt];
#pragma unroll
    for (int u = 0; u < kStageIt; u++) {
      const int q = tid + u * kWave * kColsPerBlock;
      const int j = q / kColsPerBlock, c = q - j * kColsPerBlock;
      const int i = i0 + c;
      st[u] = (q < total && i < nx) ? src[(long)j * nx + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kStageIt; u++) {
      const int q = tid + u * kWave * kColsPerBlock;
      const int j = q / kColsPerBlock, c = q - j * kColsPerBlock;
      if (q < total) T[j * kTS + c] = st[u];
    }
  }
  __syncthreads();
  const int col = i0 + wv;
  if (col < nx) {
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) {
      int p = lane * NC + c;
      v[c] = p < ny ? T[p * kTS + wv] : 0.0;
    }
    const long lb = (long)col * ny;
    line_solve_blocked<NC>(v, NC, gp(FR) + lb, gp(FG) + lb, ny, lane);
#pragma unroll
    for (int c = 0; c < NC; c++) {
      int p = lane * NC + c;
      if (p < ny) T[p * kTS + wv] = v[c];
    }
  }
  __syncthreads();
  unsigned long long mx = 0;
  for (int q = tid; q < total; q += kWave * kColsPerBlock) {
    int j = q / kColsPerBlock, c = q - j * kColsPerBlock;
    int i = i0 + c;
    if (i >= nx) continue;
    long idx = (long)j * nx + i;
    double g = T[j * kTS + c];
    if (mode == 0) {
      dst[idx] = g;
    } else if (mode == 2) {
      Unext[idx] = g;
      Gold[idx] = g;
    } else {
      double un = F[idx] + (g - Gold[idx]);
      unsigned long long bits = abs_bits(un - Unext[idx]);
      mx = bits > mx ? bits : mx;
      Unext[idx] = un;
      Gold[idx] = g;
    }
  }
  if (mode == 1) {
    mx = wave_max_u64(mx);
    if (lane == 0 && mx != 0) atomicMax(inc_bits, mx);
  }
}

// ----------------------------------------------- batched coarse sweeps ---
// Same line solves as k_coarse_x / k_coarse_y, one launch per slice index n
// over the work items of every instance; lines of different instances have
// different lengths, so the chunk count is a per-block runtime value (<= NCMAX).

template <int NCMAX>
__global__ __launch_bounds__(kWave* kRowsPerBlock) void k_coarse_xb(
    const DimInst* __restrict__ insts, const LineItem* __restrict__ items, int n, int c,
    const double* __restrict__ U_base) {
  const LineItem it = items[blockIdx.x];
  const DimInst& I = insts[it.inst];
  if (I.active && !I.active[I.idx]) return;
  if (n >= I.N || c >= I.cs) return;
  const int nx = I.nx, ny = I.ny;
  const int lane = threadIdx.x & (kWave - 1);
  const int row = it.block * kRowsPerBlock + (threadIdx.x >> 6);
  if (row >= ny) return;  // whole wave
  const gdouble* src = c == 0 ? gp(U_base) + I.off_states + (long)n * I.npts : gp(I.tmp);
  gdouble* dst = gp(I.tmp);
  const long base = (long)row * nx;
  const int K = chunks_pow2_dev(nx);
  double v[NCMAX];
#pragma unroll
  for (int cc = 0; cc < NCMAX; cc++) {
    const int p = lane * K + cc;
    v[cc] = (cc < K && p < nx) ? src[base + p] : 0.0;
  }
  line_solve_blocked<NCMAX>(v, K, gp(I.cxR) + base, gp(I.cxG) + base, nx, lane);
#pragma unroll
  for (int cc = 0; cc < NCMAX; cc++) {
    const int p = lane * K + cc;
    if (cc < K && p < nx) dst[base + p] = v[cc];
  }
}

template <int NCMAX>
__global__ __launch_bounds__(kWave* kColsPerBlock) void k_coarse_yb(
    const DimInst* __restrict__ insts, const LineItem* __restrict__ items, int n, int c, int mode,
    const double* __restrict__ F_base, double* __restrict__ G_base, double* __restrict__ U_base,
    unsigned long long* __restrict__ inc_bits) {
  extern __shared__ double T[];  // [ny][kTS]
  const LineItem it = items[blockIdx.x];
  const DimInst& I = insts[it.inst];
  if (I.active && !I.active[I.idx]) return;  // uniform over the block
  if (n >= I.N || c >= I.cs) return;
  const int nx = I.nx, ny = I.ny;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wv = tid >> 6;
  const int i0 = it.block * kColsPerBlock;
  const int total = ny * kColsPerBlock;
  const gdouble* src = gp(I.tmp);
  {
    // all loads in flight before the first LDS store
    double st[kStageIt];
#pragma unroll
    for (int u = 0; u < kStageIt; u++) {
      const int q = tid + u * kWave * kColsPerBlock;
      const int j = q / kColsPerBlock, cc = q - j * kColsPerBlock;
      const int i = i0 + cc;
      st[u] = (q < total && i < nx) ? src[(long)j * nx + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kStageIt; u++) {
      const int q = tid + u * kWave * kColsPerBlock;
      const int j = q / kColsPerBlock, cc = q - j * kColsPerBlock;
      if (q < total) T[j * kTS + cc] = st[u];
    }
  }
  __syncthreads();
  const int col = i0 + wv;
  if (col < nx) {
    const int K = chunks_pow2_dev(ny);
    double v[NCMAX];
#pragma unroll
    for (int cc = 0; cc < NCMAX; cc++) {
      int p = lane * K + cc;
      v[cc] = (cc < K && p < ny) ? T[p * kTS + wv] : 0.0;
    }
    const long lb = (long)col * ny;
    line_solve_blocked<NCMAX>(v, K, gp(I.cyR) + lb, gp(I.cyG) + lb, ny, lane);
#pragma unroll
    for (int cc = 0; cc < NCMAX; cc++) {
      int p = lane * K + cc;
      if (cc < K && p < ny) T[p * kTS + wv] = v[cc];
    }
  }
  __syncthreads();
  const int md = (c + 1 == I.cs) ? mode : 0;
  gdouble* tmpw = gp(I.tmp);
  const gdouble* Fn = gp(F_base) + I.off_slices + (long)n * I.npts;
  gdouble* Gn = gp(G_base) + I.off_slices + (long)n * I.npts;
  gdouble* Un = gp(U_base) + I.off_states + (long)(n + 1) * I.npts;
  unsigned long long mx = 0;
  if (md == 1) {
    // correction: all loads of F, G_old and the old U in flight before use
    double fv[kStageIt], gv[kStageIt], uv[kStageIt];
#pragma unroll
    for (int u = 0; u < kStageIt; u++) {
      const int q = tid + u * kWave * kColsPerBlock;
      const int j = q / kColsPerBlock, cc = q - j * kColsPerBlock;
      const int i = i0 + cc;
      const bool ok = q < total && i < nx;
      const long idx = ok ? (long)j * nx + i : 0;
      fv[u] = ok ? Fn[idx] : 0.0;
      gv[u] = ok ? Gn[idx] : 0.0;
      uv[u] = ok ? Un[idx] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kStageIt; u++) {
      const int q = tid + u * kWave * kColsPerBlock;
      const int j = q / kColsPerBlock, cc = q - j * kColsPerBlock;
      const int i = i0 + cc;
      if (q < total && i < nx) {
        const long idx = (long)j * nx + i;
        const double g = T[j * kTS + cc];
        const double un = fv[u] + (g - gv[u]);
        const unsigned long long bits = abs_bits(un - uv[u]);
        mx = bits > mx ? bits : mx;
        Un[idx] = un;
        Gn[idx] = g;
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < kStageIt; u++) {
      const int q = tid + u * kWave * kColsPerBlock;
      const int j = q / kColsPerBlock, cc = q - j * kColsPerBlock;
      const int i = i0 + cc;
      if (q < total && i < nx) {
        const long idx = (long)j * nx + i;
        const double g = T[j * kTS + cc];
        if (md == 0) {
          tmpw[idx] = g;
        } else {
          Un[idx] = g;
          Gn[idx] = g;
        }
      }
    }
  }
  if (md == 1) {
    mx = wave_max_u64(mx);
    if (lane == 0 && mx != 0) atomicMax(inc_bits + I.idx, mx);
  }
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

int chunks_pow2(int n) {
  int c = (n + kWave - 1) / kWave, p = 1;
  while (p < c) p <<= 1;
  return p;
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

hipError_t launch_chunk_phi(const double* G, int n_lines, int n_pos, int M, double* phiC,
                            double* phiS, hipStream_t s) {
  int blocks = (n_lines + 63) / 64;
  hipLaunchKernelGGL(k_chunk_phi, dim3(blocks), dim3(64), 0, s, G, n_lines, n_pos, M, phiC, phiS);
  return hipGetLastError();
}

hipError_t launch_to_interleaved(const DimInst* d_inst, const DimInst& h, const double* U_in,
                                 hipStream_t s) {
  dim3 grid((h.nx + 63) / 64, h.ny, h.B);
  hipLaunchKernelGGL(k_to_interleaved, grid, dim3(kWave), 0, s, d_inst, U_in);
  return hipGetLastError();
}

hipError_t launch_from_interleaved(const DimInst* d_inst, const DimInst& h, double* F_out,
                                   bool with_corr, hipStream_t s) {
  dim3 grid((h.nx + 63) / 64, h.ny, h.B);
  hipLaunchKernelGGL(k_from_interleaved, grid, dim3(kWave), 0, s, d_inst, F_out, (int)with_corr);
  return hipGetLastError();
}

template <int L, int M, int DIR, bool HP, int SGN = 0>
static hipError_t launch_sweep_t(const DimInst* d_insts, const WorkItem* d_work, int n_work,
                                 int step, hipStream_t s) {
  hipLaunchKernelGGL((k_fine_sweep<L, M, DIR, HP, SGN>), dim3(n_work), dim3(kWave), 0, s, d_insts,
                     d_work, step);
  return hipGetLastError();
}

template <int L, int M>
static hipError_t launch_sweep_lm(const DimInst* d_insts, const WorkItem* d_work, int n_work,
                                  int dir, int has_prev, int step, hipStream_t s, int sgn) {
  if (sgn != 0) {  // Douglas-Rachford: x adds S, y subtracts it
    if (dir == 0)
      return has_prev ? launch_sweep_t<L, M, 0, true, 1>(d_insts, d_work, n_work, step, s)
                      : launch_sweep_t<L, M, 0, false, 1>(d_insts, d_work, n_work, step, s);
    return launch_sweep_t<L, M, 1, true, -1>(d_insts, d_work, n_work, step, s);
  }
  if (dir == 0)
    return has_prev ? launch_sweep_t<L, M, 0, true>(d_insts, d_work, n_work, step, s)
                    : launch_sweep_t<L, M, 0, false>(d_insts, d_work, n_work, step, s);
  return has_prev ? launch_sweep_t<L, M, 1, true>(d_insts, d_work, n_work, step, s)
                  : launch_sweep_t<L, M, 1, false>(d_insts, d_work, n_work, step, s);
}

template <int M>
static hipError_t launch_sweep_m(const DimInst* d_insts, const WorkItem* d_work, int n_work, int L,
                                 int dir, int has_prev, int step, hipStream_t s, int sgn) {
  switch (L) {
    case 8: return launch_sweep_lm<8, M>(d_insts, d_work, n_work, dir, has_prev, step, s, sgn);
    case 16: return launch_sweep_lm<16, M>(d_insts, d_work, n_work, dir, has_prev, step, s, sgn);
    case 32: return launch_sweep_lm<32, M>(d_insts, d_work, n_work, dir, has_prev, step, s, sgn);
    case 64: return launch_sweep_lm<64, M>(d_insts, d_work, n_work, dir, has_prev, step, s, sgn);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fine_sweep(const DimInst* d_insts, const WorkItem* d_work, int n_work, int L,
                             int M, int dir, int has_prev, int step, hipStream_t s, int sgn) {
  switch (M) {
    case 16: return launch_sweep_m<16>(d_insts, d_work, n_work, L, dir, has_prev, step, s, sgn);
    case 32: return launch_sweep_m<32>(d_insts, d_work, n_work, L, dir, has_prev, step, s, sgn);
    default: return hipErrorInvalidValue;
  }
}

template <int NC>
static hipError_t launch_cx(const DimInst* d_inst, const DimInst& h, const double* src,
                            double* dst, bool fine, hipStream_t s) {
  hipLaunchKernelGGL((k_coarse_x<NC>), dim3((h.ny + kRowsPerBlock - 1) / kRowsPerBlock),
                     dim3(kWave * kRowsPerBlock), 0, s, d_inst, src, dst, fine ? h.fxE : h.cxE,
                     fine ? h.fxR : h.cxR, fine ? h.fxG : h.cxG);
  return hipGetLastError();
}

hipError_t launch_coarse_x(const DimInst* d_inst, const DimInst& h, const double* src, double* dst,
                           bool fine, hipStream_t s) {
  switch (chunks_pow2(h.nx)) {
    case 1: return launch_cx<1>(d_inst, h, src, dst, fine, s);
    case 2: return launch_cx<2>(d_inst, h, src, dst, fine, s);
    case 4: return launch_cx<4>(d_inst, h, src, dst, fine, s);
    case 8: return launch_cx<8>(d_inst, h, src, dst, fine, s);
    case 16: return launch_cx<16>(d_inst, h, src, dst, fine, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NC>
static hipError_t launch_cy(const DimInst* d_inst, const DimInst& h, const double* src,
                            double* dst, int mode, const double* F, double* G_old,
                            double* U_next, unsigned long long* inc_bits, bool fine,
                            hipStream_t s) {
  size_t lds = (size_t)h.ny * kTS * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_coarse_y<NC>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kMaxCoarseLine * kTS * (int)sizeof(double));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_coarse_y<NC>), dim3((h.nx + kColsPerBlock - 1) / kColsPerBlock),
                     dim3(kWave * kColsPerBlock), lds, s, d_inst, src, dst, mode, F, G_old, U_next,
                     inc_bits, fine ? h.fyE : h.cyE, fine ? h.fyR : h.cyR, fine ? h.fyG : h.cyG);
  return hipGetLastError();
}

hipError_t launch_coarse_y(const DimInst* d_inst, const DimInst& h, const double* src, double* dst,
                           int mode, const double* F, double* G_old, double* U_next,
                           unsigned long long* inc_bits, bool fine, hipStream_t s) {
  switch (chunks_pow2(h.ny)) {
    case 1: return launch_cy<1>(d_inst, h, src, dst, mode, F, G_old, U_next, inc_bits, fine, s);
    case 2: return launch_cy<2>(d_inst, h, src, dst, mode, F, G_old, U_next, inc_bits, fine, s);
    case 4: return launch_cy<4>(d_inst, h, src, dst, mode, F, G_old, U_next, inc_bits, fine, s);
    case 8: return launch_cy<8>(d_inst, h, src, dst, mode, F, G_old, U_next, inc_bits, fine, s);
    case 16: return launch_cy<16>(d_inst, h, src, dst, mode, F, G_old, U_next, inc_bits, fine, s);
    default: return hipErrorInvalidValue;
  }
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
                            int c, const double* U_base, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_coarse_xb<16>), dim3(n_items), dim3(kWave * kRowsPerBlock), 0, s, d_insts,
                     items, n, c, U_base);
  return hipGetLastError();
}

hipError_t launch_coarse_yb(const DimInst* d_insts, const LineItem* items, int n_items, int n,
                            int c, int mode, const double* F_base, double* G_base, double* U_base,
                            unsigned long long* inc_bits, int max_ny, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_coarse_yb<16>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kMaxCoarseLine * kTS * (int)sizeof(double));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  size_t lds = (size_t)max_ny * kTS * sizeof(double);
  hipLaunchKernelGGL((k_coarse_yb<16>), dim3(n_items), dim3(kWave * kColsPerBlock), lds, s,
                     d_insts, items, n, c, mode, F_base, G_base, U_base, inc_bits);
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
