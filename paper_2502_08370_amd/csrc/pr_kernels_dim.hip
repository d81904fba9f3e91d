// HIP kernels (gfx950, wave64, FP64) for the dimensional-splitting FIE
// propagators of parareal with splitting (arXiv 2502.08370, section 2.2
// eq. FIE_method; section 3 for the propagators and the parareal update).
//
// Every substep (I - tau A_dir) V = U is a set of independent tridiagonal
// line solves (section 2.2, last paragraphs). The matrices do not change in
// time, so each line's LU factorisation is computed once per tau and reused
// by every slice and every step.
#include "pr_internal.h"

#include <cfloat>

namespace prk {

namespace {

constexpr int kWave = 64;

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
  double u_prev = 1.0;
  double wl = job.tau_over_h2 * face[0];
  for (int p = 0; p < job.n_pos; p++) {
    double wr = job.tau_over_h2 * face[(long)(p + 1) * job.face_pos_stride];
    double diag = 1.0 + wl + wr + job.react;
    double e = (p == 0) ? 0.0 : wl / u_prev;
    double u = diag - wl * e;
    double r = 1.0 / u;
    double g = (p + 1 < job.n_pos) ? wr * r : 0.0;
    long idx = job.pos_major ? (long)p * job.n_lines + line : (long)line * job.n_pos + p;
    job.E[idx] = e;
    job.R[idx] = r;
    job.G[idx] = g;
    u_prev = u;
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
  double* Zb = I.Z + b * I.slab + ((long)j * nx + i0) * L;
  const int cnt = min(64, nx - i0);
  for (int q = lane; q < cnt * L; q += kWave) {
    int t = q / L, s = q - t * L;
    Zb[q] = tile[s][t];
  }
}

// Z (+ the pending chunk correction of the last y sweep) -> natural F[slice][j][i].
__global__ __launch_bounds__(kWave) void k_from_interleaved(const DimInst* __restrict__ insts,
                                                            double* __restrict__ F) {
  __shared__ double tile[64][65];
  const DimInst& I = insts[0];
  const int lane = threadIdx.x;
  const int i0 = blockIdx.x * 64, j = blockIdx.y, b = blockIdx.z;
  const int L = I.L, nx = I.nx, M = I.M, Py = I.Py;
  const long npts = (long)nx * I.ny;
  const double* Zb = I.Z + b * I.slab + ((long)j * nx + i0) * L;
  const double* sig = I.sigY + (long)b * nx * Py * L;
  const int cnt = min(64, nx - i0);
  const int kj = j / M;
  for (int q = lane; q < cnt * L; q += kWave) {
    int t = q / L, s = q - t * L;
    int i = i0 + t;
    double phi = I.fyPhiC[(long)j * nx + i];
    double sg = sig[((long)i * Py + kj) * L + s];
    tile[s][t] = fma(phi, sg, Zb[q]);
  }
  __syncthreads();
  for (int s = 0; s < L; s++) {
    int slice = b * L + s;
    if (slice < I.N && lane < cnt) F[slice * npts + (long)j * nx + i0 + lane] = tile[s][lane];
  }
}

// -------------------------------------------------------- fine sweeps ---

// One substep of the fine FIE step for every line of direction `dir` of every
// slice of the work items' instances. Lanes = (line in group, slice); each
// wave walks its lines position by position in chunks of M, keeping the
// chunk in registers. If has_prev, the pending chunk correction of the
// previous (other-direction) sweep is added to every value on load.
template <int L, int M>
__global__ __launch_bounds__(kWave) void k_fine_sweep(const DimInst* __restrict__ insts,
                                                      const WorkItem* __restrict__ work, int dir,
                                                      int has_prev, int step) {
  constexpr int G = kWave / L;            // lines per wave
  constexpr int NQ = (G * M + kWave - 1) / kWave;
  __shared__ double sE[G][M + 1], sR[G][M + 1], sG[G][M + 1], sP[G][M + 1];

  const WorkItem w = work[blockIdx.x];
  const DimInst& I = insts[w.inst];
  if (step >= I.steps) return;  // this instance has finished its fine steps
  const int lane = threadIdx.x;
  const int gsub = lane / L;
  const int sl = lane - gsub * L;

  int n_lines, n_pos, P, Pprev;
  long lstr, pstr;
  const double *E, *R, *Gf, *phiPrev, *phiS, *sigPrev;
  double* sigOut;
  if (dir == 0) {
    n_lines = I.ny; n_pos = I.nx; P = I.Px; Pprev = I.Py;
    lstr = (long)I.nx * L; pstr = L;
    E = I.fxE; R = I.fxR; Gf = I.fxG; phiS = I.fxPhiS;
    phiPrev = I.fyPhiC;
    sigPrev = I.sigY + (long)w.b * I.nx * I.Py * L;
    sigOut = I.sigX + (long)w.b * I.ny * I.Px * L;
  } else {
    n_lines = I.nx; n_pos = I.ny; P = I.Py; Pprev = I.Px;
    lstr = L; pstr = (long)I.nx * L;
    E = I.fyE; R = I.fyR; Gf = I.fyG; phiS = I.fyPhiS;
    phiPrev = I.fxPhiC;
    sigPrev = I.sigX + (long)w.b * I.ny * I.Px * L;
    sigOut = I.sigY + (long)w.b * I.nx * I.Py * L;
  }
  const int line0 = w.group * G;
  const int line = line0 + gsub;
  const bool active = line < n_lines;
  const int lc = active ? line : n_lines - 1;   // clamped for in-bounds loads
  const int kprev = lc / M;
  double* zbase = I.Z + w.b * I.slab + (long)lc * lstr + sl;

  double ycarry = 0.0;
  for (int k = 0; k < P; k++) {
    const int p0 = k * M;
    const int cnt = min(M, n_pos - p0);
    // stage this chunk's factors (shared by the L lanes of each line) in LDS
#pragma unroll
    for (int qq = 0; qq < NQ; qq++) {
      int q = lane + qq * kWave;
      if (q < G * M) {
        int g = q / M, t = q - g * M;
        int ln = line0 + g, p = p0 + t;
        bool ok = ln < n_lines && p < n_pos;
        long idx = (long)(ok ? ln : 0) * n_pos + (ok ? p : 0);
        sE[g][t] = ok ? E[idx] : 0.0;
        sR[g][t] = ok ? R[idx] : 0.0;
        sG[g][t] = ok ? Gf[idx] : 0.0;
        sP[g][t] = (ok && has_prev) ? phiPrev[idx] : 0.0;
      }
    }
    double v[M];
#pragma unroll
    for (int t = 0; t < M; t++) {
      int p = p0 + (t < cnt ? t : 0);
      v[t] = zbase[(long)p * pstr];
    }
    double sg[M];
    if (has_prev) {
#pragma unroll
      for (int t = 0; t < M; t++) {
        int p = p0 + (t < cnt ? t : 0);
        sg[t] = sigPrev[((long)p * Pprev + kprev) * L + sl];
      }
    }
    __syncthreads();
    // forward elimination (carried across chunks)
    double y = ycarry;
#pragma unroll
    for (int t = 0; t < M; t++) {
      if (t < cnt) {
        double d = has_prev ? fma(sP[gsub][t], sg[t], v[t]) : v[t];
        y = fma(sE[gsub][t], y, d);
        v[t] = y;
      }
    }
    ycarry = y;
    // back substitution inside the chunk with a zero carry past its end
    double z = 0.0;
#pragma unroll
    for (int t = M - 1; t >= 0; t--) {
      if (t < cnt) {
        z = fma(sG[gsub][t], z, sR[gsub][t] * v[t]);
        v[t] = z;
      }
    }
    if (active) {
#pragma unroll
      for (int t = 0; t < M; t++)
        if (t < cnt) zbase[(long)(p0 + t) * pstr] = v[t];
      sigOut[((long)line * P + k) * L + sl] = v[0];  // first value, resolved below
    }
    __syncthreads();
  }
  // carries: sigma_{P-1} = 0, sigma_k = zfirst_{k+1} + phi_{k+1 start} sigma_{k+1}
  if (active) {
    double* so = sigOut + (long)line * P * L + sl;
    double sigma = 0.0;
    double zf_next = so[(long)(P - 1) * L];
    so[(long)(P - 1) * L] = 0.0;
    for (int k = P - 2; k >= 0; k--) {
      sigma = fma(phiS[(long)line * P + k + 1], sigma, zf_next);
      zf_next = so[(long)k * L];
      so[(long)k * L] = sigma;
    }
  }
}

// -------------------------------------------------------- coarse sweeps ---
// One state (natural layout), lane = line. These solve each line exactly
// (no deferred correction): the coarse chain is serial in the slices, so the
// result must be final when the next slice starts.

constexpr int kCT = 32;  // columns per LDS tile of the coarse x sweep

// x-lines (rows): lane = row, the strided direction goes through an LDS
// transpose so that global loads and stores stay coalesced.
__global__ __launch_bounds__(kWave) void k_coarse_x(const DimInst* __restrict__ insts,
                                                    const double* __restrict__ src,
                                                    double* __restrict__ dst) {
  __shared__ double T[kWave][kCT + 1];
  const DimInst& I = insts[0];
  const int nx = I.nx, ny = I.ny;
  const int lane = threadIdx.x;
  const int j0 = blockIdx.x * kWave;
  const int row = j0 + lane;
  const bool active = row < ny;
  const int rc = active ? row : ny - 1;
  const int ntile = (nx + kCT - 1) / kCT;
  // forward elimination, tile by tile
  double y = 0.0;
  for (int tI = 0; tI < ntile; tI++) {
    const int i0 = tI * kCT, cnt = min(kCT, nx - i0);
    for (int q = lane; q < kWave * kCT; q += kWave) {
      int r = q / kCT, c = q - r * kCT;
      int rr = j0 + r;
      if (rr < ny && c < cnt) T[r][c] = src[(long)rr * nx + i0 + c];
    }
    double e[kCT];
#pragma unroll
    for (int t = 0; t < kCT; t++) e[t] = (t < cnt) ? I.cxE[(long)(i0 + t) * ny + rc] : 0.0;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kCT; t++) {
      if (t < cnt) {
        y = fma(e[t], y, T[lane][t]);
        T[lane][t] = y;
      }
    }
    __syncthreads();
    for (int q = lane; q < kWave * kCT; q += kWave) {
      int r = q / kCT, c = q - r * kCT;
      int rr = j0 + r;
      if (rr < ny && c < cnt) dst[(long)rr * nx + i0 + c] = T[r][c];
    }
    __syncthreads();
  }
  // back substitution, tiles in reverse
  double x = 0.0;
  for (int tI = ntile - 1; tI >= 0; tI--) {
    const int i0 = tI * kCT, cnt = min(kCT, nx - i0);
    for (int q = lane; q < kWave * kCT; q += kWave) {
      int r = q / kCT, c = q - r * kCT;
      int rr = j0 + r;
      if (rr < ny && c < cnt) T[r][c] = dst[(long)rr * nx + i0 + c];
    }
    double rv[kCT], gv[kCT];
#pragma unroll
    for (int t = 0; t < kCT; t++) {
      rv[t] = (t < cnt) ? I.cxR[(long)(i0 + t) * ny + rc] : 0.0;
      gv[t] = (t < cnt) ? I.cxG[(long)(i0 + t) * ny + rc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = kCT - 1; t >= 0; t--) {
      if (t < cnt) {
        x = fma(gv[t], x, rv[t] * T[lane][t]);
        T[lane][t] = x;
      }
    }
    __syncthreads();
    for (int q = lane; q < kWave * kCT; q += kWave) {
      int r = q / kCT, c = q - r * kCT;
      int rr = j0 + r;
      if (rr < ny && c < cnt) dst[(long)rr * nx + i0 + c] = T[r][c];
    }
    __syncthreads();
  }
}

constexpr int kRY = 16;  // rows per register batch of the coarse y sweep

// y-lines (columns): lane = column, naturally coalesced.
__global__ __launch_bounds__(kWave) void k_coarse_y(const DimInst* __restrict__ insts,
                                                    const double* __restrict__ src,
                                                    double* __restrict__ dst, int mode,
                                                    const double* __restrict__ F,
                                                    double* __restrict__ Gold,
                                                    double* __restrict__ Unext,
                                                    unsigned long long* __restrict__ inc_bits) {
  const DimInst& I = insts[0];
  const int nx = I.nx, ny = I.ny;
  const int col = blockIdx.x * kWave + threadIdx.x;
  const bool active = col < nx;
  const int cc = active ? col : nx - 1;
  const int nb = (ny + kRY - 1) / kRY;
  double y = 0.0;
  for (int bI = 0; bI < nb; bI++) {
    const int jb = bI * kRY, cnt = min(kRY, ny - jb);
    double d[kRY], e[kRY];
#pragma unroll
    for (int t = 0; t < kRY; t++) {
      int j = jb + (t < cnt ? t : 0);
      d[t] = src[(long)j * nx + cc];
      e[t] = I.cyE[(long)j * nx + cc];
    }
#pragma unroll
    for (int t = 0; t < kRY; t++) {
      if (t < cnt) {
        y = fma(e[t], y, d[t]);
        d[t] = y;
      }
    }
    if (active) {
#pragma unroll
      for (int t = 0; t < kRY; t++)
        if (t < cnt) dst[(long)(jb + t) * nx + cc] = d[t];
    }
  }
  double x = 0.0;
  unsigned long long mx = 0;
  for (int bI = nb - 1; bI >= 0; bI--) {
    const int jb = bI * kRY, cnt = min(kRY, ny - jb);
    double v[kRY], rv[kRY], gv[kRY];
#pragma unroll
    for (int t = 0; t < kRY; t++) {
      int j = jb + (t < cnt ? t : 0);
      long idx = (long)j * nx + cc;
      v[t] = dst[idx];
      rv[t] = I.cyR[idx];
      gv[t] = I.cyG[idx];
    }
#pragma unroll
    for (int t = kRY - 1; t >= 0; t--) {
      if (t < cnt) {
        x = fma(gv[t], x, rv[t] * v[t]);
        v[t] = x;
      }
    }
    if (!active) continue;
    if (mode == 0) {
#pragma unroll
      for (int t = 0; t < kRY; t++)
        if (t < cnt) dst[(long)(jb + t) * nx + cc] = v[t];
    } else if (mode == 2) {
#pragma unroll
      for (int t = 0; t < kRY; t++)
        if (t < cnt) {
          long idx = (long)(jb + t) * nx + cc;
          Unext[idx] = v[t];
          Gold[idx] = v[t];
        }
    } else {
      double f[kRY], go[kRY], uo[kRY];
#pragma unroll
      for (int t = 0; t < kRY; t++) {
        int j = jb + (t < cnt ? t : 0);
        long idx = (long)j * nx + cc;
        f[t] = F[idx];
        go[t] = Gold[idx];
        uo[t] = Unext[idx];
      }
#pragma unroll
      for (int t = 0; t < kRY; t++)
        if (t < cnt) {
          long idx = (long)(jb + t) * nx + cc;
          double un = f[t] + (v[t] - go[t]);
          unsigned long long bits = abs_bits(un - uo[t]);
          mx = bits > mx ? bits : mx;
          Unext[idx] = un;
          Gold[idx] = v[t];
        }
    }
  }
  if (mode == 1) {
    mx = wave_max_u64(mx);
    if (threadIdx.x == 0 && mx != 0) atomicMax(inc_bits, mx);
  }
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
                                   hipStream_t s) {
  dim3 grid((h.nx + 63) / 64, h.ny, h.B);
  hipLaunchKernelGGL(k_from_interleaved, grid, dim3(kWave), 0, s, d_inst, F_out);
  return hipGetLastError();
}

template <int L, int M>
static hipError_t launch_sweep_t(const DimInst* d_insts, const WorkItem* d_work, int n_work,
                                 int dir, int has_prev, int step, hipStream_t s) {
  hipLaunchKernelGGL((k_fine_sweep<L, M>), dim3(n_work), dim3(kWave), 0, s, d_insts, d_work, dir,
                     has_prev, step);
  return hipGetLastError();
}

template <int M>
static hipError_t launch_sweep_m(const DimInst* d_insts, const WorkItem* d_work, int n_work, int L,
                                 int dir, int has_prev, int step, hipStream_t s) {
  switch (L) {
    case 1: return launch_sweep_t<1, M>(d_insts, d_work, n_work, dir, has_prev, step, s);
    case 2: return launch_sweep_t<2, M>(d_insts, d_work, n_work, dir, has_prev, step, s);
    case 4: return launch_sweep_t<4, M>(d_insts, d_work, n_work, dir, has_prev, step, s);
    case 8: return launch_sweep_t<8, M>(d_insts, d_work, n_work, dir, has_prev, step, s);
    case 16: return launch_sweep_t<16, M>(d_insts, d_work, n_work, dir, has_prev, step, s);
    case 32: return launch_sweep_t<32, M>(d_insts, d_work, n_work, dir, has_prev, step, s);
    case 64: return launch_sweep_t<64, M>(d_insts, d_work, n_work, dir, has_prev, step, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fine_sweep(const DimInst* d_insts, const WorkItem* d_work, int n_work, int L,
                             int M, int dir, int has_prev, int step, hipStream_t s) {
  switch (M) {
    case 16: return launch_sweep_m<16>(d_insts, d_work, n_work, L, dir, has_prev, step, s);
    case 32: return launch_sweep_m<32>(d_insts, d_work, n_work, L, dir, has_prev, step, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_coarse_x(const DimInst* d_inst, const DimInst& h, const double* src, double* dst,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_x, dim3((h.ny + kWave - 1) / kWave), dim3(kWave), 0, s, d_inst, src,
                     dst);
  return hipGetLastError();
}

hipError_t launch_coarse_y(const DimInst* d_inst, const DimInst& h, const double* src, double* dst,
                           int mode, const double* F, double* G_old, double* U_next,
                           unsigned long long* inc_bits, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_y, dim3((h.nx + kWave - 1) / kWave), dim3(kWave), 0, s, d_inst, src,
                     dst, mode, F, G_old, U_next, inc_bits);
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

}  // namespace prk
