// HIP kernels of the 2D domain-decomposition split into vertical strips
// (arXiv 2502.08370, section 2.1: L_k u = div(rho_k D grad u) - rho_k c u with a
// partition of unity rho_k of overlapping strips; eq. FIE_method for the
// substeps). Each strip system is solved exactly by block cyclic reduction in
// y; the set-up kernels precompute every block the solve needs, the solve
// kernels stream those blocks through the FP64 matrix cores with all slices as
// the columns of the product.
#include "pr_internal.h"

#include <algorithm>
#include <climits>

namespace prk {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// ------------------------------------------------------------------ set-up ---

// Flux weights of node (i, r) for colour weights rho (half grid of x): west and
// east x-faces (rho on the face), south and north y-faces (rho at the node).
struct Flux {
  double w, e, s, n, react;
};

__device__ inline Flux node_flux(const DD2Geo& g, int i, int r) {
  Flux f;
  const double rn = g.rho[2 * i + 1];
  f.w = g.tx * g.rho[2 * i] * g.ax[(long)r * (g.nx + 1) + i];
  f.e = g.tx * g.rho[2 * i + 2] * g.ax[(long)r * (g.nx + 1) + i + 1];
  f.s = g.ty * rn * g.ay[(long)r * g.nx + i];
  f.n = g.ty * rn * g.ay[(long)(r + 1) * g.nx + i];
  f.react = g.tc * rn;
  return f;
}

// Entry (o, k) of the level-0 diagonal block D_r = I - tau A restricted to block
// row r (tridiagonal in x); identity on the padding o >= w.
__device__ inline double d0_entry(const DD2Geo& g, int r, int o, int k) {
  if (o >= g.w || k >= g.w) return o == k ? 1.0 : 0.0;
  const int d = k - o;
  if (d < -1 || d > 1) return 0.0;
  const Flux f = node_flux(g, g.col0 + o, r);
  if (d == 0) return 1.0 + f.w + f.e + f.s + f.n + f.react;
  return d < 0 ? -f.w : -f.e;
}

__global__ void k_dd2_bc(DD2Geo g, double* __restrict__ bc) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)g.ny * g.W) return;
  const int r = (int)(t / g.W), o = (int)(t % g.W);
  double b = 0.0, c = 0.0;
  if (o < g.w) {
    const Flux f = node_flux(g, g.col0 + o, r);
    if (r > 0) b = -f.s;
    if (r + 1 < g.ny) c = -f.n;
  }
  bc[((long)r * 2 + 0) * g.W + o] = b;
  bc[((long)r * 2 + 1) * g.W + o] = c;
}

// Inverses of the level-0 blocks, which are tridiagonal: one LU (pivots and
// multipliers, a short recurrence in LDS) per block, then one Thomas solve per
// column of the identity, thread per column (for a fixed row the threads write
// consecutive entries). The inverse lands in columns [W, 2W) of the matrix at
// aug + m * mstride (row stride 2W), where the level-1 set-up reads it; the LU
// itself (multipliers m, reciprocal pivots ip, back factors g = -sup * ip) is
// kept at tri + 3 W m for the level-0 solves.
__global__ __launch_bounds__(256) void k_dd2_tri_inv(DD2Geo g, double* __restrict__ aug,
                                                     long mstride, double* __restrict__ tri) {
  __shared__ double piv[kDD2MaxW], mul[kDD2MaxW], sup[kDD2MaxW];
  const int m = blockIdx.x, r = 2 * m, W = g.W, LD = 2 * W;
  double* A = aug + m * mstride + W;
  for (int o = threadIdx.x; o < W; o += blockDim.x) {
    piv[o] = d0_entry(g, r, o, o);                         // diagonal
    mul[o] = o > 0 ? d0_entry(g, r, o, o - 1) : 0.0;       // sub-diagonal
    sup[o] = o + 1 < W ? d0_entry(g, r, o, o + 1) : 0.0;   // super-diagonal
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int o = 1; o < W; o++) {
      const double f = mul[o] / piv[o - 1];
      mul[o] = f;
      piv[o] = piv[o] - f * sup[o - 1];
    }
  __syncthreads();
  double* T = tri + (long)m * 3 * W;
  for (int o = threadIdx.x; o < W; o += blockDim.x) {
    const double ip = 1.0 / piv[o];
    T[o] = mul[o];
    T[W + o] = ip;
    T[2 * W + o] = -sup[o] * ip;
  }
  for (int j = threadIdx.x; j < W; j += blockDim.x) {
    double y = 0.0;
    for (int o = 0; o < W; o++) {  // forward: L y = e_j
      y = (o == j) ? 1.0 : (o > j ? -mul[o] * y : 0.0);
      A[(long)o * LD + j] = y;
    }
    double x = 0.0;
    for (int o = W - 1; o >= 0; o--) {  // back: U x = y
      x = (A[(long)o * LD + j] - sup[o] * x) / piv[o];
      A[(long)o * LD + j] = x;
    }
  }
}

// Gauss-Jordan elimination without pivoting (the blocks are strictly
// diagonally dominant M-matrices at every level of the reduction), one
// workgroup per matrix, in panels of np pivots: the panel's rows P are reduced
// among themselves in LDS (P <- B^-1 P, B their pivot block), then every other
// row q takes row_q -= f_q P with f_q its panel-column values before the panel
// (so the panel columns of row q vanish and the result equals np single
// steps), one pass over the matrix per panel. Columns left of the panel are
// finished unit columns and are never read again.
__global__ __launch_bounds__(512) void k_dd2_gj(double* __restrict__ aug, long mstride, int W,
                                                int LD, int np_max) {
  extern __shared__ double lds[];
  double* panel = lds;                      // [np_max][LD]
  double* fq = lds + (long)np_max * LD;     // [np_max][W]
  double* A = aug + blockIdx.x * mstride;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int p0 = 0; p0 < W; p0 += np_max) {
    const int np = min(np_max, W - p0), span = LD - p0;
    for (int e = tid; e < np * span; e += nt) {
      const int j = e / span, c = p0 + e % span;
      panel[j * LD + c] = A[(long)(p0 + j) * LD + c];
    }
    for (int e = tid; e < W * np; e += nt) {
      const int q = e / np, j = e % np;
      fq[j * W + q] = A[(long)q * LD + p0 + j];
    }
    __syncthreads();
    for (int t = 0; t < np; t++) {
      const double inv = 1.0 / panel[t * LD + p0 + t];
      __syncthreads();
      for (int c = p0 + tid; c < LD; c += nt) panel[t * LD + c] *= inv;
      __syncthreads();
      for (int e = tid; e < (np - 1) * span; e += nt) {
        int j = e / span;
        j += (j >= t);
        const int c = p0 + e % span;
        if (c != p0 + t) panel[j * LD + c] -= panel[j * LD + p0 + t] * panel[t * LD + c];
      }
      __syncthreads();
      if (tid < np && tid != t) panel[tid * LD + p0 + t] = 0.0;
      __syncthreads();
    }
    for (int e = tid; e < W * span; e += nt) {
      const int q = e / span, c = p0 + e % span;
      double v;
      if (q >= p0 && q < p0 + np) {
        v = panel[(q - p0) * LD + c];
      } else {
        v = A[(long)q * LD + c];
        for (int t = 0; t < np; t++) v -= fq[t * W + q] * panel[t * LD + c];
      }
      A[(long)q * LD + c] = v;
    }
    __syncthreads();
  }
}

// Level-0 kept row r = 2a + 1 reduced onto level 1:
//   D' = D_r - b_r Dinv_{r-1} c_{r-1} - c_r Dinv_{r+1} b_{r+1}
//   B' = -b_r Dinv_{r-1} b_{r-1},  C' = -c_r Dinv_{r+1} c_{r+1}
// (diagonal couplings as row / column scalings of the dense inverses).
__global__ void k_dd2_scale0(DD2Geo g, const double* __restrict__ bc,
                             const double* __restrict__ aug0, long mstride, double* __restrict__ Dn,
                             double* __restrict__ Bn, double* __restrict__ Cn) {
  const int a = blockIdx.y, r = 2 * a + 1, W = g.W;
  const bool up = r + 1 < g.ny;
  const double* Im = aug0 + (long)(r / 2) * mstride + W;   // Dinv of row r - 1 (ld 2W)
  const double* Ip = aug0 + (long)((r + 1) / 2) * mstride + W;
  const double* b_r = bc + ((long)r * 2 + 0) * W;
  const double* c_r = bc + ((long)r * 2 + 1) * W;
  const double* b_m = bc + ((long)(r - 1) * 2 + 0) * W;
  const double* c_m = bc + ((long)(r - 1) * 2 + 1) * W;
  const double* b_p = up ? bc + ((long)(r + 1) * 2 + 0) * W : nullptr;
  const double* c_p = up ? bc + ((long)(r + 1) * 2 + 1) * W : nullptr;
  const long base = (long)a * W * W;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)W * W;
       t += (long)gridDim.x * blockDim.x) {
    const int o = (int)(t / W), k = (int)(t % W);
    const double im = Im[(long)o * 2 * W + k];
    double d = d0_entry(g, r, o, k) - b_r[o] * im * c_m[k];
    double bb = -(b_r[o] * im * b_m[k]);
    double cc = 0.0;
    if (up) {
      const double ip = Ip[(long)o * 2 * W + k];
      d = d - c_r[o] * ip * b_p[k];
      cc = -(c_r[o] * ip * c_p[k]);
    }
    Dn[base + t] = d;
    Bn[base + t] = bb;
    Cn[base + t] = cc;
  }
}

__global__ void k_dd2_aug(const double* __restrict__ D, const double* __restrict__ B,
                          const double* __restrict__ C, int W, double* __restrict__ aug) {
  const int e = blockIdx.y, a = 2 * e;
  const int LD = 4 * W;
  const long src = (long)a * W * W;
  double* A = aug + (long)e * W * LD;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)W * LD;
       t += (long)gridDim.x * blockDim.x) {
    const int o = (int)(t / LD), col = (int)(t % LD);
    const int part = col / W, k = col % W;
    double v;
    if (part == 0)
      v = D[src + (long)o * W + k];
    else if (part == 1)
      v = (o == k) ? 1.0 : 0.0;
    else if (part == 2)
      v = B[src + (long)o * W + k];
    else
      v = C[src + (long)o * W + k];
    A[t] = v;
  }
}

// C = base + sgn * A B over W x W blocks: 64 x 64 output tile per workgroup,
// 4 x 4 per thread (rows ty + 16 i, columns tx + 16 j), k in LDS panels of 16.
__global__ __launch_bounds__(256) void k_dd2_gemm(const DD2Gemm* __restrict__ jobs, int W) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const DD2Gemm J = jobs[blockIdx.y];
  const int tiles = (W + 63) / 64;
  const int o0 = (blockIdx.x / tiles) * 64, c0 = (blockIdx.x % tiles) * 64;
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < W; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int kk = e % 16, oo = e / 16;  // A tile: consecutive threads walk k
      const int o = o0 + oo;
      As[kk][oo] = o < W ? J.A[(long)o * J.lda + k0 + kk] : 0.0;
      const int cc = e % 64, kb = e / 64;  // B tile: consecutive threads walk columns
      const int c = c0 + cc;
      Bs[kb][cc] = c < W ? J.B[(long)(k0 + kb) * J.ldb + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk++) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; i++) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; j++) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int o = o0 + ty + 16 * i, c = c0 + tx + 16 * j;
      if (o < W && c < W) {
        const double b = J.base ? J.base[(long)o * J.ldbase + c] : 0.0;
        J.C[(long)o * J.ldc + c] = b + J.sgn * acc[i][j];
      }
    }
}

__global__ void k_dd2_store(const DD2Copy* __restrict__ jobs, int W) {
  const DD2Copy J = jobs[blockIdx.y];
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)W * W;
       t += (long)gridDim.x * blockDim.x) {
    const int o = (int)(t / W), k = (int)(t % W);
    J.dst[dd2_frag(W, o, k)] = J.src[(long)o * J.ld + k];
  }
}

// ------------------------------------------------------------------- solve ---

// Solve phase kernel. A unit's output is rows [16 mb0, 16 (mb0 + nmb)) of block
// row U.row against TN tiles of 16 slice columns starting at b0:
//   APPLY: Y[row] = A0 Z[row]
//   KUP:   Z[row] = Z[row] - A1 Y[rowm] - A2 Y[rowp]
//   BACK:  Z[row] = Y[row] - A1 Z[rowm] - A2 Z[rowp]
// v_mfma_f64_16x16x4: lane l supplies A[l % 16][l / 16] and X[l / 16][l % 16]
// and holds D[4 v + l / 16][l % 16] in accumulator register v. Pool matrices
// are stored in exactly that A order, so each (k-block, row tile) fragment is
// one contiguous 512-byte load. Inputs past the strip width are read at the
// last column (finite values) and meet zero matrix entries. Single-state solves
// (Npad = 1) feed zeros into the 15 unused columns.
// KSPLIT = 0: one block row per workgroup, wave i taking its row tiles
// [RT i, RT i + RT) (the waves share the row's right-hand sides through the CU's
// cache). KSPLIT = 1: four units per workgroup, one per wave. KSPLIT = 4, 8 or
// 16: one unit per workgroup, the k-blocks dealt to KSPLIT waves and the partial
// products summed through LDS in a tree (KSPLIT times shorter dependent chains
// for launches with few units). The loads of the next k-blocks are issued
// before the products of the current one.

// k-blocks loaded ahead of the one being multiplied, in the whole-row launches
// (KSPLIT = 0) and in the others (measured: three in the whole-row launches
// cost more registers than they hide).
constexpr int kRowPrefetch = 2;
constexpr int kSplitPrefetch = 2;

// Workgroup size of a solve launch: whole-row launches hold up to 32 row tiles
// (W <= 512), RT per wave; split launches one wave per k-range share.
template <int KSPLIT>
constexpr int solve_threads() {
  return KSPLIT == 0 ? kWave * (32 / kDD2WholeRowTiles) : (KSPLIT == 1 ? 4 * kWave : KSPLIT * kWave);
}

template <int MODE, int TN, int RT>
struct Frag {
  double a[RT];
  double x[TN];
};

// Loads of k-block kb (clamped into [0, kb_end) so every address is valid; a
// block past the end, or a row tile past nmb, contributes a zero A fragment).
template <int MODE, int TN, int RT, bool SINGLE, bool NT>
__device__ __forceinline__ void load_frag(Frag<MODE, TN, RT>& f, const double* A, long mbW,
                                          const double* X, int kb, int kb_end, int kq, int cl,
                                          int w, int nmb, int Npad) {
  const bool live = kb < kb_end;
  kb = min(kb, kb_end - 1);
  const int k = min(kb * 4 + kq, w - 1);
#pragma unroll
  for (int r = 0; r < RT; r++) {
    // the factor stream is read once (non-temporal where measured faster: launches
    // without split-K; the split ones read their blocks in shorter pieces)
    f.a[r] = (live && r < nmb) ? (NT ? __builtin_nontemporal_load(&A[((long)kb * mbW + r) * 64])
                                     : A[((long)kb * mbW + r) * 64]) : 0.0;
  }
#pragma unroll
  for (int nt = 0; nt < TN; nt++) {
    const long xo = SINGLE ? (long)k : (long)k * Npad + nt * 16;
    const double v = X[xo];
    f.x[nt] = (SINGLE && cl != 0) ? 0.0 : v;
  }
}

template <int MODE, int TN, bool SINGLE, int KSPLIT>
__global__ __launch_bounds__(solve_threads<KSPLIT>()) void k_dd2_solve(
    const DD2Unit* __restrict__ units, int n_units, const double* __restrict__ pool,
    double* __restrict__ Z, double* __restrict__ Y, int nx, int Npad, int b0) {
  // row tiles per wave
  constexpr int RT = KSPLIT == 0 ? kDD2WholeRowTiles : kDD2SplitTiles;
  const int lane = threadIdx.x % kWave;
  // the wave index is uniform across the wave: say so, so that the unit's fields
  // live in scalar registers and its guards are scalar branches
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int u = KSPLIT == 1 ? blockIdx.x * 4 + wave : blockIdx.x;
  if (u >= n_units) return;  // no barrier follows for KSPLIT <= 1; split units are whole workgroups
  const DD2Unit U = units[u];
  const int W = U.W, w = U.w;
  // KSPLIT = 0: the unit is a whole block row; wave i takes its row tiles [RT i, RT i + RT)
  const int mb0 = KSPLIT == 0 ? U.mb0 + RT * wave : U.mb0;
  const int nmb = KSPLIT == 0 ? min(RT, U.nmb - RT * wave) : U.nmb;
  if (nmb <= 0) return;
  const long mbW = W >> 4;
  const int nkb = W >> 2;
  const int kq = lane >> 4, cl = lane & 15;
  // this wave's k-blocks
  const int kb_lo = KSPLIT <= 1 ? 0 : (nkb * wave) / KSPLIT;
  const int kb_hi = KSPLIT <= 1 ? nkb : (nkb * (wave + 1)) / KSPLIT;
  d4 acc[RT][TN];
#pragma unroll
  for (int r = 0; r < RT; r++)
#pragma unroll
    for (int nt = 0; nt < TN; nt++) acc[r][nt] = d4{0.0, 0.0, 0.0, 0.0};
  const long col_off = SINGLE ? 0 : (long)b0 + cl;
  constexpr int n_terms = (MODE == DD2_KUP || MODE == DD2_BACK) ? 2 : 1;
#pragma unroll 1
  for (int term = 0; term < n_terms; term++) {
    long aoff;
    int rx;
    if (MODE == DD2_APPLY) {
      aoff = U.A0; rx = U.row;
    } else {
      aoff = term == 0 ? U.A1 : U.A2;
      rx = term == 0 ? U.rowm : U.rowp;
    }
    if (rx < 0 || kb_lo >= kb_hi) continue;
    const double* Xb = (MODE == DD2_KUP) ? Y : Z;
    const double* A = pool + aoff + (long)mb0 * 64 + lane;
    const double* X = Xb + ((long)rx * nx + U.col0) * Npad + col_off;
    // ring of PF k-blocks in flight ahead of the one being multiplied
    constexpr int PF = KSPLIT == 0 ? kRowPrefetch : kSplitPrefetch;
    Frag<MODE, TN, RT> ring[PF + 1];
#pragma unroll
    for (int q = 0; q < PF; q++)
      load_frag<MODE, TN, RT, SINGLE, (KSPLIT <= 1)>(ring[q], A, mbW, X, kb_lo + q, kb_hi, kq, cl, w, nmb, Npad);
    for (int kb = kb_lo; kb < kb_hi; kb++) {
      if (kb + PF < kb_hi)
        load_frag<MODE, TN, RT, SINGLE, (KSPLIT <= 1)>(ring[PF], A, mbW, X, kb + PF, kb_hi, kq, cl, w, nmb, Npad);
#pragma unroll
      for (int r = 0; r < RT; r++) {
        if (r < nmb) {
#pragma unroll
          for (int nt = 0; nt < TN; nt++)
            acc[r][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ring[0].a[r], ring[0].x[nt], acc[r][nt], 0, 0, 0);
        }
      }
#pragma unroll
      for (int q = 0; q < PF; q++) ring[q] = ring[q + 1];
    }
  }
  if (KSPLIT > 1) {
    // tree over the waves: at each stage waves [half, 2 half) leave their
    // partial products in LDS and waves [0, half) add them
    constexpr int kSlots = KSPLIT > 1 ? KSPLIT / 2 : 1;
    __shared__ double part[kSlots * RT * TN * 4 * kWave];
#pragma unroll 1
    for (int half = KSPLIT / 2; half >= 1; half >>= 1) {
      if (wave >= half && wave < 2 * half) {
#pragma unroll
        for (int r = 0; r < RT; r++)
#pragma unroll
          for (int nt = 0; nt < TN; nt++)
#pragma unroll
            for (int v = 0; v < 4; v++)
              part[((((wave - half) * RT + r) * TN + nt) * 4 + v) * kWave + lane] = acc[r][nt][v];
      }
      __syncthreads();
      if (wave < half) {
#pragma unroll
        for (int r = 0; r < RT; r++)
#pragma unroll
          for (int nt = 0; nt < TN; nt++)
#pragma unroll
            for (int v = 0; v < 4; v++)
              acc[r][nt][v] += part[(((wave * RT + r) * TN + nt) * 4 + v) * kWave + lane];
      }
      __syncthreads();
    }
    if (wave > 0) return;
  }
#pragma unroll
  for (int r = 0; r < RT; r++) {
    if (r >= nmb) continue;
#pragma unroll
    for (int nt = 0; nt < TN; nt++)
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int o = (mb0 + r) * 16 + 4 * v + kq;
        if (o >= w || (SINGLE && cl != 0)) continue;
        const long idx = ((long)U.row * nx + U.col0 + o) * Npad + (SINGLE ? 0 : b0 + nt * 16 + cl);
        const double val = acc[r][nt][v];
        if (MODE == DD2_APPLY)
          Y[idx] = val;
        else if (MODE == DD2_KUP)
          Z[idx] = Z[idx] - val;
        else
          Z[idx] = Y[idx] - val;
      }
  }
}

// Level-0 kept rows: Z[row] -= b_row Y[rowm] + c_row Y[rowp], one workgroup per row.
__global__ void k_dd2_kup0(const DD2Row* __restrict__ rows, const double* __restrict__ bcp,
                           double* __restrict__ Z, const double* __restrict__ Y, int nx,
                           int Npad) {
  const DD2Row R = rows[blockIdx.x];
  const double* vb = bcp + R.bc;
  const double* vc = bcp + R.bc + R.W;
  const long n = (long)R.w * Npad;
  const long base = ((long)R.row * nx + R.col0) * Npad;
  const long bm = ((long)R.rowm * nx + R.col0) * Npad;
  const long bp = R.rowp >= 0 ? ((long)R.rowp * nx + R.col0) * Npad : -1;
  for (long t = threadIdx.x; t < n; t += blockDim.x) {
    const int o = (int)(t / Npad);
    double v = Z[base + t] - vb[o] * Y[bm + t];
    if (bp >= 0) v = v - vc[o] * Y[bp + t];
    Z[base + t] = v;
  }
}

// Level-0 eliminated rows: D_r is tridiagonal in x, so its solves are Thomas
// sweeps with the stored LU (z_o = rhs_o - m_o z_{o-1}, then
// x_o = ip_o z_o + g_o x_{o+1}) along each line (row, slice column):
//   BACK = false: Y[r] = D_r^-1 Z[r]
//   BACK = true:  Z[r] = Y[r] - D_r^-1 (b_r Z[r-1] + c_r Z[r+1])
// A missing neighbour row reads y of the row itself against a zero coupling.

// One lane per line: the row is walked in chunks of kTriChunk positions whose
// loads are issued together; the forward values are stored in the output row
// and read back by the backward sweep of the same lane. The lanes of a row read
// the same LU entries (one request per wave and address).
constexpr int kTriChunk = 16;

template <bool BACK>
__global__ __launch_bounds__(64) void k_dd2_tri0(const DD2Row* __restrict__ rows, int n_rows,
                                                 const double* __restrict__ tri,
                                                 const double* __restrict__ bcp,
                                                 double* __restrict__ Z, double* __restrict__ Y,
                                                 int nx, int Npad) {
  const long t = blockIdx.x * (long)kWave + threadIdx.x;
  if (t >= (long)n_rows * Npad) return;
  const DD2Row R = rows[t / Npad];
  const int b = (int)(t % Npad), w = R.w;
  const long sp = Npad;  // stride between consecutive columns of a row
  const double* fm = tri + R.tri;
  const double* fip = fm + R.W;
  const double* fg = fm + 2 * R.W;
  const long own = ((long)R.row * nx + R.col0) * Npad + b;
  double* out = (BACK ? Z : Y) + own;
  const double* src = Z + own;     // forward input without coupling (BACK = false)
  const double* yr = Y + own;      // y of the row (BACK = true)
  const double* zm = R.rowm >= 0 ? Z + ((long)R.rowm * nx + R.col0) * Npad + b : yr;
  const double* zp = R.rowp >= 0 ? Z + ((long)R.rowp * nx + R.col0) * Npad + b : yr;
  const double* vb = bcp + R.bc;
  const double* vc = vb + R.W;
  double z = 0.0;
  for (int c0 = 0; c0 < w; c0 += kTriChunk) {
    double v[kTriChunk], mm[kTriChunk];
#pragma unroll
    for (int j = 0; j < kTriChunk; j++) {
      const int o = min(c0 + j, w - 1);  // clamped: past the end nothing is stored
      mm[j] = fm[o];
      v[j] = BACK ? vb[o] * zm[o * sp] + vc[o] * zp[o * sp] : src[o * sp];
    }
#pragma unroll
    for (int j = 0; j < kTriChunk; j++) {
      z = v[j] - mm[j] * z;
      if (c0 + j < w) out[(c0 + j) * sp] = z;
    }
  }
  double x = 0.0;
  for (int c1 = w; c1 > 0; c1 -= kTriChunk) {  // positions c1 - 1, c1 - 2, ...
    double zz[kTriChunk], ii[kTriChunk], gg[kTriChunk], yy[kTriChunk];
#pragma unroll
    for (int j = 0; j < kTriChunk; j++) {
      const int o = max(c1 - 1 - j, 0);
      zz[j] = out[o * sp];
      ii[j] = fip[o];
      gg[j] = fg[o];
      yy[j] = BACK ? yr[o * sp] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kTriChunk; j++) {
      x = ii[j] * zz[j] + gg[j] * x;
      if (c1 - 1 - j >= 0) out[(c1 - 1 - j) * sp] = BACK ? yy[j] - x : x;
    }
  }
}

// Staged in LDS, for all slice columns: one workgroup per (row, group of 16
// columns). The row's right-hand sides (w x 16, coalesced rows of 128 bytes)
// and LU land in LDS; wave v takes columns 4v..4v+3 with 16 lanes per column,
// lane q holding the segment [qK, qK + K) of the row; each sweep composes the
// segment's affine maps, scans them over the 16 lanes and re-runs the segment
// from its incoming value; the result leaves through LDS. The tile is stored
// column by column with an odd column stride and K is odd, so that the lanes of
// a wave (16 segments x 4 columns, or 16 columns x 4 positions when loading)
// fall on different LDS banks.
constexpr int kTriStageMaxW = 512;

__host__ __device__ inline int tri0s_stride(int w) { return w | 1; }
__host__ __device__ inline size_t tri0s_lds_bytes(int wmax) {
  return ((size_t)16 * tri0s_stride(wmax) + 3 * (size_t)wmax) * sizeof(double);
}

template <bool BACK>
__global__ __launch_bounds__(256) void k_dd2_tri0s(const DD2Row* __restrict__ rows,
                                                   const double* __restrict__ tri,
                                                   const double* __restrict__ bcp,
                                                   double* __restrict__ Z, double* __restrict__ Y,
                                                   int nx, int Npad) {
  extern __shared__ double lds[];
  const DD2Row R = rows[blockIdx.x];
  const int b0 = (int)blockIdx.y * 16;
  const int w = R.w, tid = threadIdx.x;
  const int S = tri0s_stride(w);
  double* T = lds;                     // [16][S]: column c at T + c S
  double* Fm = lds + 16 * S;           // [w] multipliers
  double* Fi = Fm + w;                 // [w] reciprocal pivots
  double* Fg = Fi + w;                 // [w] back factors
  const double* fm = tri + R.tri;
  const long own = ((long)R.row * nx + R.col0) * Npad + b0;
  const double* zm = Z + ((long)(R.rowm >= 0 ? R.rowm : R.row) * nx + R.col0) * Npad + b0;
  const double* zp = Z + ((long)(R.rowp >= 0 ? R.rowp : R.row) * nx + R.col0) * Npad + b0;
  const double* vb = bcp + R.bc;
  const double* vc = vb + R.W;
  // right-hand sides and LU into LDS (a missing neighbour row meets a zero coupling)
  const int n = w * 16;
  constexpr int U = BACK ? 8 : 16;
  for (int e0 = tid; e0 < n; e0 += U * 256) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int e = min(e0 + u * 256, n - 1);
      const int p = e >> 4, c = e & 15;
      v[u] = BACK ? vb[p] * zm[(long)p * Npad + c] + vc[p] * zp[(long)p * Npad + c]
                  : Z[own + (long)p * Npad + c];
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int e = e0 + u * 256;
      if (e < n) T[(e & 15) * S + (e >> 4)] = v[u];
    }
  }
  for (int p = tid; p < w; p += 256) {
    Fm[p] = fm[p];
    Fi[p] = fm[R.W + p];
    Fg[p] = fm[2 * R.W + p];
  }
  __syncthreads();
  const int lane = tid % kWave, q = lane & 15;
  const int c = (tid / kWave) * 4 + (lane >> 4);
  const int K = ((w + 15) >> 4) | 1;
  const int p0 = min(q * K, w), p1 = min(p0 + K, w);
  double* Tc = T + c * S;
  // forward: z_p = v_p - m_p z_{p-1}
  double A = 1.0, B = 0.0;
#pragma unroll 4
  for (int p = p0; p < p1; p++) {
    const double m = Fm[p];
    B = fma(-m, B, Tc[p]);
    A = -m * A;
  }
#pragma unroll
  for (int d = 1; d < 16; d <<= 1) {
    const double ap = __shfl_up(A, d, 16);
    const double bp = __shfl_up(B, d, 16);
    if (q >= d) {
      B = fma(A, bp, B);
      A = A * ap;
    }
  }
  double z = __shfl_up(B, 1, 16);
  if (q == 0) z = 0.0;
#pragma unroll 4
  for (int p = p0; p < p1; p++) {
    z = fma(-Fm[p], z, Tc[p]);
    Tc[p] = z;
  }
  // backward: x_p = ip_p z_p + g_p x_{p+1}
  A = 1.0;
  B = 0.0;
#pragma unroll 4
  for (int p = p1 - 1; p >= p0; p--) {
    const double g = Fg[p];
    B = fma(g, B, Fi[p] * Tc[p]);
    A = g * A;
  }
#pragma unroll
  for (int d = 1; d < 16; d <<= 1) {
    const double an = __shfl_down(A, d, 16);
    const double bn = __shfl_down(B, d, 16);
    if (q + d < 16) {
      B = fma(A, bn, B);
      A = A * an;
    }
  }
  double x = __shfl_down(B, 1, 16);
  if (q == 15) x = 0.0;
#pragma unroll 4
  for (int p = p1 - 1; p >= p0; p--) {
    x = fma(Fg[p], x, Fi[p] * Tc[p]);
    Tc[p] = x;
  }
  __syncthreads();
  double* out = (BACK ? Z : Y) + own;
  const double* yr = Y + own;
  constexpr int V = 8;
  for (int e0 = tid; e0 < n; e0 += V * 256) {
    double yv[V];
#pragma unroll
    for (int u = 0; u < V; u++) {
      const int e = min(e0 + u * 256, n - 1);
      yv[u] = BACK ? yr[(long)(e >> 4) * Npad + (e & 15)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < V; u++) {
      const int e = e0 + u * 256;
      if (e >= n) continue;
      const double v = T[(e & 15) * S + (e >> 4)];
      out[(long)(e >> 4) * Npad + (e & 15)] = BACK ? yv[u] - v : v;
    }
  }
}

// Inclusive scans over the 64 lanes of the affine maps v -> a v + b: upwards
// lane i ends with f_i o ... o f_0, downwards with f_i o f_{i+1} o ... o f_63.
__device__ __forceinline__ void tri_scan_up(double& a, double& b, int lane) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const double ap = __shfl_up(a, off, kWave);
    const double bp = __shfl_up(b, off, kWave);
    if (lane >= off) {
      b = fma(a, bp, b);
      a = a * ap;
    }
  }
}

__device__ __forceinline__ void tri_scan_down(double& a, double& b, int lane) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const double an = __shfl_down(a, off, kWave);
    const double bn = __shfl_down(b, off, kWave);
    if (lane + off < kWave) {
      b = fma(a, bn, b);
      a = a * an;
    }
  }
}

// One wave per line: lane l holds positions [l K, l K + K) in registers (all
// loads of the line in flight together). Each sweep composes the lane's affine
// maps, scans them over the lanes to get the value entering the lane, and
// re-runs its positions from it. Positions past the row end carry zero maps
// (m = ip = g = 0), and g = 0 at the last position, so nothing crosses the end.
template <bool BACK, int K>
__global__ __launch_bounds__(256) void k_dd2_tri0w(const DD2Row* __restrict__ rows, int n_lines,
                                                   const double* __restrict__ tri,
                                                   const double* __restrict__ bcp,
                                                   double* __restrict__ Z, double* __restrict__ Y,
                                                   int nx, int Npad) {
  const int lane = threadIdx.x % kWave;
  const int line = (int)blockIdx.x * (blockDim.x / kWave) +
                   __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (line >= n_lines) return;
  const DD2Row R = rows[line / Npad];
  const int b = line % Npad, w = R.w;
  const long sp = Npad;
  const double* fm = tri + R.tri;
  const double* fip = fm + R.W;
  const double* fg = fm + 2 * R.W;
  const long own = ((long)R.row * nx + R.col0) * Npad + b;
  double* out = (BACK ? Z : Y) + own;
  const double* src = Z + own;
  const double* yr = Y + own;
  const double* zm = R.rowm >= 0 ? Z + ((long)R.rowm * nx + R.col0) * Npad + b : yr;
  const double* zp = R.rowp >= 0 ? Z + ((long)R.rowp * nx + R.col0) * Npad + b : yr;
  const double* vb = bcp + R.bc;
  const double* vc = vb + R.W;
  double v[K], mm[K], ii[K], gg[K], yy[K];
#pragma unroll
  for (int j = 0; j < K; j++) {
    const int p = lane * K + j;
    const bool in = p < w;
    const int pc = in ? p : w - 1;  // loads stay unconditional and in range
    const double m = fm[pc], ip = fip[pc], g = fg[pc];
    const double r = BACK ? vb[pc] * zm[pc * sp] + vc[pc] * zp[pc * sp] : src[pc * sp];
    const double y = BACK ? yr[pc * sp] : 0.0;
    mm[j] = in ? m : 0.0;
    ii[j] = in ? ip : 0.0;
    gg[j] = in ? g : 0.0;
    v[j] = in ? r : 0.0;
    yy[j] = y;
  }
  // forward: z_p = v_p - m_p z_{p-1}
  double A = 1.0, B = 0.0;
#pragma unroll
  for (int j = 0; j < K; j++) {
    B = fma(-mm[j], B, v[j]);
    A = -mm[j] * A;
  }
  tri_scan_up(A, B, lane);
  double z = __shfl_up(B, 1, kWave);
  if (lane == 0) z = 0.0;
#pragma unroll
  for (int j = 0; j < K; j++) {
    z = fma(-mm[j], z, v[j]);
    v[j] = z;
  }
  // backward: x_p = ip_p z_p + g_p x_{p+1}
  A = 1.0;
  B = 0.0;
#pragma unroll
  for (int j = K - 1; j >= 0; j--) {
    B = fma(gg[j], B, ii[j] * v[j]);
    A = gg[j] * A;
  }
  tri_scan_down(A, B, lane);
  double x = __shfl_down(B, 1, kWave);
  if (lane == kWave - 1) x = 0.0;
#pragma unroll
  for (int j = K - 1; j >= 0; j--) {
    x = fma(gg[j], x, ii[j] * v[j]);
    const int p = lane * K + j;
    if (p < w) out[p * sp] = BACK ? yy[j] - x : x;
  }
}

// [N][npts] -> [npts][Npad] through a 64 x 64 LDS tile (rows: slices, columns: points).
__global__ void k_dd2_to_sm(const double* __restrict__ U, double* __restrict__ Zs, long npts,
                            int N, int Npad) {
  __shared__ double tile[64][65];
  const long p0 = blockIdx.x * 64L;
  const int b0 = blockIdx.y * 64;
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
  for (int bb = ty; bb < 64; bb += blockDim.x / 64) {
    const int b = b0 + bb;
    const long p = p0 + tx;
    tile[bb][tx] = (b < N && p < npts) ? U[(long)b * npts + p] : 0.0;
  }
  __syncthreads();
  for (int pp = ty; pp < 64; pp += blockDim.x / 64) {
    const long p = p0 + pp;
    const int b = b0 + tx;
    if (p < npts && b < Npad) Zs[p * Npad + b] = tile[tx][pp];
  }
}

__global__ void k_dd2_from_sm(const double* __restrict__ Zs, double* __restrict__ U, long npts,
                              int N, int Npad) {
  __shared__ double tile[64][65];
  const long p0 = blockIdx.x * 64L;
  const int b0 = blockIdx.y * 64;
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
  for (int pp = ty; pp < 64; pp += blockDim.x / 64) {
    const long p = p0 + pp;
    const int b = b0 + tx;
    tile[pp][tx] = (p < npts && b < Npad) ? Zs[p * Npad + b] : 0.0;
  }
  __syncthreads();
  for (int bb = ty; bb < 64; bb += blockDim.x / 64) {
    const int b = b0 + bb;
    const long p = p0 + tx;
    if (b < N && p < npts) U[(long)b * npts + p] = tile[tx][bb];
  }
}

__global__ void k_dd2_force_sm(const double* __restrict__ fS, const double* __restrict__ gtab,
                               long gstride, int steps, int t, double* __restrict__ Zs, long npts,
                               int N, int Npad) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= npts * Npad) return;
  const long p = e / Npad;
  const int b = (int)(e % Npad);
  if (b >= N) return;
  double v = Zs[e];
#pragma unroll
  for (int m = 0; m < kMaxForcing; m++)
    v = fma(gtab[m * gstride + (long)b * steps + t], fS[m * npts + p], v);
  Zs[e] = v;
}

// Douglas-Rachford terms of the strip split: S = tau A_k U for colour k's
// weights over the whole grid (zero off the colour's support), slice-minor
// [node][Npad] (Npad = 1: one state in natural layout). A_k is the operator of
// the set-up kernels: x-fluxes weighted by rho on the face, y-fluxes and the
// reaction by rho at the node column.
__global__ void k_dd2_stencil(DD2Geo g, const double* __restrict__ U, double* __restrict__ S,
                              int Npad) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long npts = (long)g.nx * g.ny;
  if (e >= npts * Npad) return;
  const long p = e / Npad;
  const int i = (int)(p % g.nx), k = (int)(p / g.nx);
  const Flux f = node_flux(g, i, k);
  const double u = U[e];
  const double uw = i > 0 ? U[e - Npad] : 0.0;
  const double ue = i + 1 < g.nx ? U[e + Npad] : 0.0;
  const double us = k > 0 ? U[e - (long)g.nx * Npad] : 0.0;
  const double un = k + 1 < g.ny ? U[e + (long)g.nx * Npad] : 0.0;
  S[e] = f.w * (uw - u) + f.e * (ue - u) + f.s * (us - u) + f.n * (un - u) - f.react * u;
}

__global__ void k_dd2_axpy(double* __restrict__ Z, const double* __restrict__ S, double a,
                           long n) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < n) Z[e] = fma(a, S[e], Z[e]);
}

unsigned grid_for(long n, int per_block, unsigned cap = 65535u) {
  long g = (n + per_block - 1) / per_block;
  return (unsigned)std::max<long>(1, std::min<long>(g, cap));
}

}  // namespace

// ------------------------------------------------------------- launchers ---

hipError_t launch_dd2_bc(const DD2Geo& g, double* bc, hipStream_t s) {
  hipLaunchKernelGGL(k_dd2_bc, dim3(grid_for((long)g.ny * g.W, 256, 1u << 30)), dim3(256), 0, s,
                     g, bc);
  return hipGetLastError();
}

hipError_t launch_dd2_gj(double* aug, long mstride, int n, int W, int LD, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (W > kDD2MaxW || LD > 4 * kDD2MaxW) return hipErrorInvalidValue;
  // panel of up to 8 pivots within ~96 KB of LDS (panel rows + multipliers)
  const int np_max = std::max(1, std::min(8, (96 * 1024) / (8 * (LD + W))));
  const size_t lds = (size_t)np_max * (LD + W) * sizeof(double);
  hipLaunchKernelGGL(k_dd2_gj, dim3(n), dim3(512), lds, s, aug, mstride, W, LD, np_max);
  return hipGetLastError();
}

hipError_t launch_dd2_tri_inv(const DD2Geo& g, int n, double* aug, long mstride, double* tri,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (g.W > kDD2MaxW) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dd2_tri_inv, dim3(n), dim3(256), 0, s, g, aug, mstride, tri);
  return hipGetLastError();
}

hipError_t launch_dd2_scale0(const DD2Geo& g, const double* bc, const double* aug0, long mstride,
                             double* Dn, double* Bn, double* Cn, hipStream_t s) {
  const int n = g.ny / 2;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dd2_scale0, dim3(grid_for((long)g.W * g.W, 256, 256), n), dim3(256), 0, s,
                     g, bc, aug0, mstride, Dn, Bn, Cn);
  return hipGetLastError();
}

hipError_t launch_dd2_aug(const double* D, const double* B, const double* C, int nE, int W,
                          double* aug, hipStream_t s) {
  if (nE <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dd2_aug, dim3(grid_for((long)W * 4 * W, 256, 256), nE), dim3(256), 0, s,
                     D, B, C, W, aug);
  return hipGetLastError();
}

hipError_t launch_dd2_gemm(const DD2Gemm* jobs, int n, int W, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int tiles = (W + 63) / 64;
  hipLaunchKernelGGL(k_dd2_gemm, dim3(tiles * tiles, n), dim3(256), 0, s, jobs, W);
  return hipGetLastError();
}

hipError_t launch_dd2_store(const DD2Copy* jobs, int n, int W, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dd2_store, dim3(grid_for((long)W * W, 256, 256), n), dim3(256), 0, s, jobs,
                     W);
  return hipGetLastError();
}

namespace {
template <int MODE, bool SINGLE, int KSPLIT>
hipError_t solve_tn(int tn, const DD2Unit* units, int n_units, const double* pool, double* Z,
                    double* Y, int nx, int Npad, int b0, int waves, hipStream_t s) {
  const dim3 grid(KSPLIT == 1 ? (n_units + 3) / 4 : n_units),
      block(KSPLIT == 0 ? kWave * waves : solve_threads<KSPLIT>());
  if constexpr (KSPLIT == 16) {
    // sixteen waves leave 128 registers per lane and 160 KB of LDS: enough for
    // at most two column tiles; wider launches split eight ways
    if (tn > 2) return solve_tn<MODE, SINGLE, 8>(tn, units, n_units, pool, Z, Y, nx, Npad, b0, 0, s);
    if (tn == 1)
      hipLaunchKernelGGL((k_dd2_solve<MODE, 1, SINGLE, 16>), grid, block, 0, s, units, n_units, pool, Z, Y, nx, Npad, b0);
    else
      hipLaunchKernelGGL((k_dd2_solve<MODE, 2, SINGLE, 16>), grid, block, 0, s, units, n_units, pool, Z, Y, nx, Npad, b0);
    return hipGetLastError();
  } else {
    switch (tn) {
      case 1: hipLaunchKernelGGL((k_dd2_solve<MODE, 1, SINGLE, KSPLIT>), grid, block, 0, s, units, n_units, pool, Z, Y, nx, Npad, b0); break;
      case 2: hipLaunchKernelGGL((k_dd2_solve<MODE, 2, SINGLE, KSPLIT>), grid, block, 0, s, units, n_units, pool, Z, Y, nx, Npad, b0); break;
      case 3: hipLaunchKernelGGL((k_dd2_solve<MODE, 3, SINGLE, KSPLIT>), grid, block, 0, s, units, n_units, pool, Z, Y, nx, Npad, b0); break;
      default: hipLaunchKernelGGL((k_dd2_solve<MODE, 4, SINGLE, KSPLIT>), grid, block, 0, s, units, n_units, pool, Z, Y, nx, Npad, b0); break;
    }
    return hipGetLastError();
  }
}

template <int MODE, int KSPLIT>
hipError_t solve_mode(const DD2Unit* units, int n_units, const double* pool, double* Z,
                      double* Y, int nx, int Npad, bool single, int waves, hipStream_t s) {
  if (single)
    return solve_tn<MODE, true, KSPLIT>(1, units, n_units, pool, Z, Y, nx, 1, 0, waves, s);
  for (int b0 = 0; b0 < Npad; b0 += 64) {
    const int tn = std::min(4, (Npad - b0) / 16);
    hipError_t e = solve_tn<MODE, false, KSPLIT>(tn, units, n_units, pool, Z, Y, nx, Npad, b0,
                                                 waves, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int KSPLIT>
hipError_t solve_split(int mode, const DD2Unit* units, int n_units, const double* pool,
                       double* Z, double* Y, int nx, int Npad, bool single, int waves,
                       hipStream_t s) {
  switch (mode) {
    case DD2_APPLY: return solve_mode<DD2_APPLY, KSPLIT>(units, n_units, pool, Z, Y, nx, Npad, single, waves, s);
    case DD2_KUP: return solve_mode<DD2_KUP, KSPLIT>(units, n_units, pool, Z, Y, nx, Npad, single, waves, s);
    case DD2_BACK: return solve_mode<DD2_BACK, KSPLIT>(units, n_units, pool, Z, Y, nx, Npad, single, waves, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

hipError_t launch_dd2_solve(int mode, const DD2Unit* units, int n_units, const double* pool,
                            double* Z, double* Y, int nx, int Npad, bool single, int split,
                            int waves, hipStream_t s) {
  if (n_units <= 0) return hipSuccess;
  if (!single && Npad % 16 != 0) return hipErrorInvalidValue;
  if (split == 16) return solve_split<16>(mode, units, n_units, pool, Z, Y, nx, Npad, single, 0, s);
  if (split == 8) return solve_split<8>(mode, units, n_units, pool, Z, Y, nx, Npad, single, 0, s);
  if (split == 4) return solve_split<4>(mode, units, n_units, pool, Z, Y, nx, Npad, single, 0, s);
  if (split == 0) {
    if (waves < 1 || waves * kDD2WholeRowTiles > 32) return hipErrorInvalidValue;
    return solve_split<0>(mode, units, n_units, pool, Z, Y, nx, Npad, single, waves, s);
  }
  return solve_split<1>(mode, units, n_units, pool, Z, Y, nx, Npad, single, 0, s);
}

hipError_t launch_dd2_kup0(const DD2Row* rows, int n_rows, const double* bc, double* Z,
                           const double* Y, int nx, int Npad, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dd2_kup0, dim3(n_rows), dim3(256), 0, s, rows, bc, Z, Y, nx, Npad);
  return hipGetLastError();
}

namespace {
template <bool BACK>
hipError_t tri0_wave(int K, const DD2Row* rows, int n_lines, const double* tri, const double* bc,
                     double* Z, double* Y, int nx, int Npad, hipStream_t s) {
  const dim3 grid((unsigned)((n_lines + 3) / 4)), block(4 * kWave);
  switch (K) {
    case 1: hipLaunchKernelGGL((k_dd2_tri0w<BACK, 1>), grid, block, 0, s, rows, n_lines, tri, bc, Z, Y, nx, Npad); break;
    case 2: hipLaunchKernelGGL((k_dd2_tri0w<BACK, 2>), grid, block, 0, s, rows, n_lines, tri, bc, Z, Y, nx, Npad); break;
    case 4: hipLaunchKernelGGL((k_dd2_tri0w<BACK, 4>), grid, block, 0, s, rows, n_lines, tri, bc, Z, Y, nx, Npad); break;
    case 8: hipLaunchKernelGGL((k_dd2_tri0w<BACK, 8>), grid, block, 0, s, rows, n_lines, tri, bc, Z, Y, nx, Npad); break;
    case 16: hipLaunchKernelGGL((k_dd2_tri0w<BACK, 16>), grid, block, 0, s, rows, n_lines, tri, bc, Z, Y, nx, Npad); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_dd2_tri0(bool back, const DD2Row* rows, int n_rows, int wmax, bool per_line,
                           const double* tri, const double* bc, double* Z, double* Y, int nx,
                           int Npad, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  if (Npad < 1 || wmax < 1 || wmax > kDD2MaxW) return hipErrorInvalidValue;
  const long lines = (long)n_rows * Npad;
  if (lines > INT_MAX) return hipErrorInvalidValue;
  if (!per_line && Npad % 16 == 0 && wmax <= kTriStageMaxW) {
    const dim3 grid((unsigned)n_rows, (unsigned)(Npad / 16)), block(256);
    const size_t lds = tri0s_lds_bytes(wmax);
    if (back)
      hipLaunchKernelGGL(k_dd2_tri0s<true>, grid, block, lds, s, rows, tri, bc, Z, Y, nx, Npad);
    else
      hipLaunchKernelGGL(k_dd2_tri0s<false>, grid, block, lds, s, rows, tri, bc, Z, Y, nx, Npad);
    return hipGetLastError();
  }
  if (per_line) {
    int K = 1;
    while (K * kWave < wmax) K *= 2;
    return back ? tri0_wave<true>(K, rows, (int)lines, tri, bc, Z, Y, nx, Npad, s)
                : tri0_wave<false>(K, rows, (int)lines, tri, bc, Z, Y, nx, Npad, s);
  }
  const dim3 grid((unsigned)((lines + kWave - 1) / kWave)), block(kWave);
  if (back)
    hipLaunchKernelGGL(k_dd2_tri0<true>, grid, block, 0, s, rows, n_rows, tri, bc, Z, Y, nx, Npad);
  else
    hipLaunchKernelGGL(k_dd2_tri0<false>, grid, block, 0, s, rows, n_rows, tri, bc, Z, Y, nx, Npad);
  return hipGetLastError();
}

hipError_t launch_dd2_to_sm(const double* U, double* Zs, long npts, int N, int Npad,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_dd2_to_sm, dim3((unsigned)((npts + 63) / 64), (Npad + 63) / 64), dim3(256),
                     0, s, U, Zs, npts, N, Npad);
  return hipGetLastError();
}

hipError_t launch_dd2_from_sm(const double* Zs, double* U, long npts, int N, int Npad,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_dd2_from_sm, dim3((unsigned)((npts + 63) / 64), (Npad + 63) / 64),
                     dim3(256), 0, s, Zs, U, npts, N, Npad);
  return hipGetLastError();
}

hipError_t launch_dd2_force_sm(const double* fS, const double* gtab, long gstride, int steps,
                               int t, double* Zs, long npts, int N, int Npad, hipStream_t s) {
  const long n = npts * Npad;
  hipLaunchKernelGGL(k_dd2_force_sm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, fS, gtab,
                     gstride, steps, t, Zs, npts, N, Npad);
  return hipGetLastError();
}

hipError_t launch_dd2_stencil(const DD2Geo& g, const double* U, double* S, int Npad,
                              hipStream_t s) {
  const long n = (long)g.nx * g.ny * Npad;
  hipLaunchKernelGGL(k_dd2_stencil, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, U, S,
                     Npad);
  return hipGetLastError();
}

hipError_t launch_dd2_axpy(double* Z, const double* S, double a, long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dd2_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Z, S, a, n);
  return hipGetLastError();
}

}  // namespace prk
