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
// restricted matrix is the exact block of the substep.
__global__ void k_dd_factorize(const double* __restrict__ w, int n,
                               const int* __restrict__ comp_lo, const int* __restrict__ comp_hi,
                               const int* __restrict__ comp_colour, int n_comps,
                               double tau_over_h2, double* __restrict__ E,
                               double* __restrict__ R, double* __restrict__ G) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_comps) return;
  const int lo = comp_lo[c], hi = comp_hi[c], k = comp_colour[c];
  const double* wk = w + (long)k * (n + 1);
  const long base = (long)k * n;
  double u_prev = 1.0;
  double wl = tau_over_h2 * wk[lo];
  for (int i = lo; i <= hi; i++) {
    double wr = tau_over_h2 * wk[i + 1];
    double diag = 1.0 + wl + wr;
    double e = (i == lo) ? 0.0 : wl / u_prev;
    double u = diag - wl * e;
    double r = 1.0 / u;
    E[base + i] = e;
    R[base + i] = r;
    G[base + i] = (i < hi) ? wr * r : 0.0;
    u_prev = u;
    wl = wr;
  }
}

// Per segment: psi (product of e over the segment), chi_i = r_i psi_i +
// g_i chi_{i+1} (chi past the end 0) and phi_i = g_i phi_{i+1} (phi past the
// end 1), with psi_i the product of e from the segment start to i.
__global__ void k_dd_segfactors(const DDSeg* __restrict__ segs, const int* __restrict__ seg_colour,
                                int n_segs, int n, const double* __restrict__ E,
                                const double* __restrict__ R, const double* __restrict__ G,
                                double* __restrict__ CHI, double* __restrict__ PHI,
                                double* __restrict__ PSIE, double* __restrict__ CHIA,
                                double* __restrict__ PHIA) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_segs) return;
  const DDSeg sg = segs[s];
  const long base = (long)seg_colour[s] * n + sg.lo;
  double p = 1.0;
  for (int t = 0; t < sg.len; t++) {  // psi kept in CHI until the backward pass
    p = p * E[base + t];
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
// Segment solves with zero carries: forward elimination (tilde y) and back
// substitution (tilde z) of each segment, in place; records tilde y at the
// segment's last node (Yb) and tilde z at its first node (Za).
template <int L>
__global__ __launch_bounds__(kWave) void k_dd_local(const DDInst* __restrict__ insts, DDFactors f,
                                                    int colour, int seg_begin, int seg_count) {
  constexpr int G = kWave / L;
  constexpr int M = kDDSeg;
  constexpr int NQ = (G * M + kWave - 1) / kWave;
  __shared__ double sE[G][M + 1], sR[G][M + 1], sG[G][M + 1];
  const DDInst& I = insts[0];
  const int lane = threadIdx.x, gsub = lane / L, sl = lane - gsub * L;
  const int b = blockIdx.y;
  const int s0 = blockIdx.x * G;
  const long cb = (long)colour * I.n;
  const gdouble* E = gp(f.E) + cb;
  const gdouble* R = gp(f.R) + cb;
  const gdouble* Gf = gp(f.G) + cb;
  // factors of the wave's segments; padded positions act as identity
#pragma unroll
  for (int qq = 0; qq < NQ; qq++) {
    const int q = lane + qq * kWave;
    if (q < G * M) {
      const int g = q / M, t = q - g * M;
      const int sidx = s0 + g;
      const DDSeg sg = I.segs[seg_begin + min(sidx, seg_count - 1)];
      const bool ok = sidx < seg_count && t < sg.len;
      const long node = sg.lo + (ok ? t : 0);
      sE[g][t] = ok ? E[node] : 1.0;
      sR[g][t] = ok ? R[node] : 0.0;
      sG[g][t] = ok ? Gf[node] : 0.0;
    }
  }
  __syncthreads();
  const int sidx = s0 + gsub;
  const bool active = sidx < seg_count;
  const int sg_i = seg_begin + (active ? sidx : seg_count - 1);
  const DDSeg sg = I.segs[sg_i];
  gdouble* zb = gp(I.Z) + b * I.slab + (long)sg.lo * L + sl;
  double v[M];
#pragma unroll
  for (int t = 0; t < M; t++) v[t] = t < sg.len ? zb[(long)t * L] : 0.0;
  double y = 0.0;
#pragma unroll
  for (int t = 0; t < M; t++) {
    y = fma(sE[gsub][t], y, v[t]);
    v[t] = y;
  }
  double z = 0.0;
#pragma unroll
  for (int t = M - 1; t >= 0; t--) {
    z = fma(sG[gsub][t], z, sR[gsub][t] * v[t]);
    v[t] = z;
  }
  if (active) {
#pragma unroll
    for (int t = 0; t < M; t++)
      if (t < sg.len) zb[(long)t * L] = v[t];
    const long bi = ((long)b * I.n_segs + sg_i) * L + sl;
    gp(I.Yb)[bi] = y;
    gp(I.Za)[bi] = v[0];
  }
}

// ------------------------------------------------------------- phase 2 ---
// Carry resolution per (component, slice): Y_s = Yb_s + psi_s Y_{s-1} over the
// component's segments (wave scans, 64 segments per step), then
// X_s = Za_s + chi_s Y_{s-1} + phi_s X_{s+1} backwards; stores
// Yin_s = Y_{s-1} and Xin_s = X_{s+1}.
__global__ __launch_bounds__(kWave) void k_dd_carries(const DDInst* __restrict__ insts,
                                                      DDFactors f,
                                                      const int* __restrict__ comp_first,
                                                      const int* __restrict__ comp_count) {
  const DDInst& I = insts[0];
  const int lane = threadIdx.x;
  const int comp = blockIdx.x;
  const int slice = blockIdx.y;  // b * L + l
  const int b = slice / I.L, sl = slice - b * I.L;
  const int first = comp_first[comp], count = comp_count[comp];
  const long sb = (long)b * I.n_segs;
  const int nch = (count + kWave - 1) / kWave;
  double carry = 0.0;
  for (int ch = 0; ch < nch; ch++) {
    const int s = first + ch * kWave + lane;
    const bool ok = s < first + count;
    const long bi = (sb + (ok ? s : first)) * I.L + sl;
    double a = ok ? f.PSIE[s] : 1.0;
    double bb = ok ? I.Yb[bi] : 0.0;
    affine_scan_up(a, bb, lane);
    const double Y = fma(a, carry, bb);
    double prev = __shfl_up(Y, 1, kWave);
    if (lane == 0) prev = carry;
    if (ok) I.Yin[bi] = prev;
    carry = lane_value(Y, kWave - 1);
  }
  carry = 0.0;
  for (int ch = nch - 1; ch >= 0; ch--) {
    const int s = first + ch * kWave + lane;
    const bool ok = s < first + count;
    const long bi = (sb + (ok ? s : first)) * I.L + sl;
    double a = ok ? f.PHIA[s] : 0.0;
    double bb = ok ? fma(f.CHIA[s], I.Yin[bi], I.Za[bi]) : 0.0;
    affine_scan_down(a, bb, lane);
    const double X = fma(a, carry, bb);
    double next = __shfl_down(X, 1, kWave);
    if (lane == kWave - 1) next = carry;
    if (ok) I.Xin[bi] = next;
    carry = lane_value(X, 0);
  }
}

// ------------------------------------------------------------- phase 3 ---
template <int L>
__global__ __launch_bounds__(kWave) void k_dd_correct(const DDInst* __restrict__ insts,
                                                      DDFactors f, int colour, int seg_begin,
                                                      int seg_count) {
  constexpr int G = kWave / L;
  constexpr int M = kDDSeg;
  const DDInst& I = insts[0];
  const int lane = threadIdx.x, gsub = lane / L, sl = lane - gsub * L;
  const int b = blockIdx.y;
  const int sidx = blockIdx.x * G + gsub;
  if (sidx >= seg_count) return;
  const int sg_i = seg_begin + sidx;
  const DDSeg sg = I.segs[sg_i];
  const long bi = ((long)b * I.n_segs + sg_i) * L + sl;
  const double yin = gp(I.Yin)[bi], xin = gp(I.Xin)[bi];
  const long cb = (long)colour * I.n + sg.lo;
  const gdouble* chi = gp(f.CHI) + cb;
  const gdouble* phi = gp(f.PHI) + cb;
  gdouble* zb = gp(I.Z) + b * I.slab + (long)sg.lo * L + sl;
#pragma unroll 8
  for (int t = 0; t < M; t++)
    if (t < sg.len) zb[(long)t * L] = fma(phi[t], xin, fma(chi[t], yin, zb[(long)t * L]));
}

// ------------------------------------------------------ parareal update ---
__global__ void k_update(const double* __restrict__ g, const double* __restrict__ F,
                         double* __restrict__ Gold, double* __restrict__ Unext, size_t n, int mode,
                         unsigned long long* __restrict__ inc_bits) {
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
    if ((threadIdx.x & (kWave - 1)) == 0 && mx != 0) atomicMax(inc_bits, mx);
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
                               const int* comp_colour, int n_comps, double tau_over_h2, double* E,
                               double* R, double* G, hipStream_t s) {
  hipLaunchKernelGGL(k_dd_factorize, dim3((n_comps + 63) / 64), dim3(64), 0, s, w, n, comp_lo,
                     comp_hi, comp_colour, n_comps, tau_over_h2, E, R, G);
  return hipGetLastError();
}

hipError_t launch_dd_segfactors(const DDSeg* segs, const int* seg_colour, int n_segs, int n,
                                const double* E, const double* R, const double* G, double* CHI,
                                double* PHI, double* PSIE, double* CHIA, double* PHIA,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_dd_segfactors, dim3((n_segs + 63) / 64), dim3(64), 0, s, segs, seg_colour,
                     n_segs, n, E, R, G, CHI, PHI, PSIE, CHIA, PHIA);
  return hipGetLastError();
}

template <int L>
static hipError_t dd_local_t(const DDInst* d, const DDInst& h, const DDFactors& f, int colour,
                             int seg_begin, int seg_count, hipStream_t s) {
  constexpr int G = kWave / L;
  dim3 grid((seg_count + G - 1) / G, h.B);
  hipLaunchKernelGGL((k_dd_local<L>), grid, dim3(kWave), 0, s, d, f, colour, seg_begin, seg_count);
  return hipGetLastError();
}

hipError_t launch_dd_local(const DDInst* d, const DDInst& h, const DDFactors& f, int colour,
                           int seg_begin, int seg_count, hipStream_t s) {
  if (seg_count <= 0) return hipSuccess;
  switch (h.L) {
    case 1: return dd_local_t<1>(d, h, f, colour, seg_begin, seg_count, s);
    case 8: return dd_local_t<8>(d, h, f, colour, seg_begin, seg_count, s);
    case 16: return dd_local_t<16>(d, h, f, colour, seg_begin, seg_count, s);
    case 32: return dd_local_t<32>(d, h, f, colour, seg_begin, seg_count, s);
    case 64: return dd_local_t<64>(d, h, f, colour, seg_begin, seg_count, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_dd_carries(const DDInst* d, const DDInst& h, const DDFactors& f,
                             const int* comp_first, const int* comp_count, int n_comps,
                             hipStream_t s) {
  if (n_comps <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dd_carries, dim3(n_comps, h.B * h.L), dim3(kWave), 0, s, d, f, comp_first,
                     comp_count);
  return hipGetLastError();
}

template <int L>
static hipError_t dd_correct_t(const DDInst* d, const DDInst& h, const DDFactors& f, int colour,
                               int seg_begin, int seg_count, hipStream_t s) {
  constexpr int G = kWave / L;
  dim3 grid((seg_count + G - 1) / G, h.B);
  hipLaunchKernelGGL((k_dd_correct<L>), grid, dim3(kWave), 0, s, d, f, colour, seg_begin,
                     seg_count);
  return hipGetLastError();
}

hipError_t launch_dd_correct(const DDInst* d, const DDInst& h, const DDFactors& f, int colour,
                             int seg_begin, int seg_count, hipStream_t s) {
  if (seg_count <= 0) return hipSuccess;
  switch (h.L) {
    case 1: return dd_correct_t<1>(d, h, f, colour, seg_begin, seg_count, s);
    case 8: return dd_correct_t<8>(d, h, f, colour, seg_begin, seg_count, s);
    case 16: return dd_correct_t<16>(d, h, f, colour, seg_begin, seg_count, s);
    case 32: return dd_correct_t<32>(d, h, f, colour, seg_begin, seg_count, s);
    case 64: return dd_correct_t<64>(d, h, f, colour, seg_begin, seg_count, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_update(const double* g, const double* F, double* G_old, double* U_next,
                         size_t n, int mode, unsigned long long* inc_bits, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(k_update, dim3(blocks), dim3(256), 0, s, g, F, G_old, U_next, n, mode,
                     inc_bits);
  return hipGetLastError();
}

}  // namespace prk
