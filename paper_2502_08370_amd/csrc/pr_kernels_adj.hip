// HIP kernels (gfx950, FP64) for the adjoint of the fine map u(T) = (F^s)^N u0
// under dimensional splitting. One FIE step (eq. FIE_method) is
// W = Bx^{-1} U, V = By^{-1} W with Bx = I - tau A_x, By = I - tau A_y, both
// symmetric, so for L = <lambda, V>:
//   mu = By^{-1} lambda, nu = Bx^{-1} mu, dL/dU = nu,
//   dL/da_f = -(tau/h^2) (mu_q - mu_p)(V_q - V_p) for a y-face f = (p, q)
//   (x-faces with nu and W), values on boundary nodes being 0.
// The line solves reuse the fine factorisations; these kernels add the face
// gradients (one thread per face, summed in step order: deterministic) and
// apply the chain rule to the nodal log coefficient.
#include "pr_internal.h"

namespace prk {

namespace {

// gax[j][f] += -coef (nu_q - nu_p)(W_q - W_p), p = (f-1, j), q = (f, j)
__global__ void k_face_grad_x(const double* __restrict__ nu, const double* __restrict__ W,
                              int nx, int ny, double coef, double* __restrict__ gax) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)ny * (nx + 1)) return;
  const int j = (int)(t / (nx + 1)), f = (int)(t - (long)j * (nx + 1));
  const long r = (long)j * nx;
  const double np = f > 0 ? nu[r + f - 1] : 0.0, nq = f < nx ? nu[r + f] : 0.0;
  const double wp = f > 0 ? W[r + f - 1] : 0.0, wq = f < nx ? W[r + f] : 0.0;
  gax[t] += -coef * (nq - np) * (wq - wp);
}

// gay[g][i] += -coef (mu_q - mu_p)(V_q - V_p), p = (i, g-1), q = (i, g)
__global__ void k_face_grad_y(const double* __restrict__ mu, const double* __restrict__ V,
                              int nx, int ny, double coef, double* __restrict__ gay) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)(ny + 1) * nx) return;
  const int g = (int)(t / nx), i = (int)(t - (long)g * nx);
  const double mp = g > 0 ? mu[(long)(g - 1) * nx + i] : 0.0;
  const double mq = g < ny ? mu[(long)g * nx + i] : 0.0;
  const double vp = g > 0 ? V[(long)(g - 1) * nx + i] : 0.0;
  const double vq = g < ny ? V[(long)g * nx + i] : 0.0;
  gay[t] += -coef * (mq - mp) * (vq - vp);
}

// grad_theta(I, J) = 1/2 e^theta(I,J) * (sum of the gradients of the faces
// touching extended node (I, J)); x-face f of row j joins (f, j+1)-(f+1, j+1),
// y-face g of column i joins (i+1, g)-(i+1, g+1).
__global__ void k_theta_chain(const double* __restrict__ theta, const double* __restrict__ gax,
                              const double* __restrict__ gay, int nx, int ny,
                              double* __restrict__ gth) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int Wd = nx + 2;
  if (t >= (long)Wd * (ny + 2)) return;
  const int J = (int)(t / Wd), I = (int)(t - (long)J * Wd);
  double s = 0.0;
  const int j = J - 1;
  if (j >= 0 && j < ny) {
    if (I <= nx) s += gax[(long)j * (nx + 1) + I];      // node is the left end of face I
    if (I >= 1) s += gax[(long)j * (nx + 1) + I - 1];   // right end of face I-1
  }
  const int i = I - 1;
  if (gay && i >= 0 && i < nx) {
    if (J <= ny) s += gay[(long)J * nx + i];            // lower end of face J
    if (J >= 1) s += gay[(long)(J - 1) * nx + i];       // upper end of face J-1
  }
  gth[t] = 0.5 * exp(theta[t]) * s;
}

// ------------------------------------------- all slices at once (batched) ---
// The per-slice reverse passes of the parallel-in-time adjoint run on the
// slice-interleaved workspaces Z[b][j][i][l] of the fine sweeps, whose values
// carry the pending chunk correction of their last sweep: the true value at
// (i, j) is Z + phi * sigma, with phi and sigma of that sweep's direction
// (x: fxPhiC[i*ny + j], sigX[b][i/M][j][l]; y: fyPhiC[j*nx + i],
// sigY[b][j/M][i][l]). A and Bst are descriptors of the adjoint workspace and
// of the recomputed forward state of the same step.
template <int DIR>
__device__ __forceinline__ double true_value(const DimInst& D, int b, int i, int j, int l) {
  if (i < 0 || i >= D.nx || j < 0 || j >= D.ny) return 0.0;  // boundary nodes are 0
  const int L = D.L, M = D.M;
  const double z = D.Z[b * D.slab + ((long)j * D.nx + i) * L + l];
  if (DIR == 0)
    return fma(D.fxPhiC[(long)i * D.ny + j],
               D.sigX[(((long)b * D.Px + i / M) * D.ny + j) * L + l], z);
  return fma(D.fyPhiC[(long)j * D.nx + i], D.sigY[(((long)b * D.Py + j / M) * D.nx + i) * L + l],
             z);
}

// g[face] += -coef * sum over slices (a_q - a_p)(w_q - w_p): a from the adjoint
// workspace A, w from the forward state Bst, both true values after a sweep of
// direction DIR. One group of L lanes (the slices of a block) per face; every
// group loops over the slice blocks, reduces over its lanes, and its first
// lane adds the sum (one writer per face: deterministic).
template <int DIR, int L>
__global__ __launch_bounds__(64) void k_grad_faces(const DimInst* __restrict__ A,
                                                   const DimInst* __restrict__ Bst, double coef,
                                                   double* __restrict__ g) {
  constexpr int G = 64 / L;
  const DimInst& a = A[0];
  const DimInst& w = Bst[0];
  const int lane = threadIdx.x, gsub = lane / L, l = lane - gsub * L;
  const long face = (long)blockIdx.x * G + gsub;
  const int nx = a.nx, ny = a.ny;
  const long nfaces = DIR == 0 ? (long)ny * (nx + 1) : (long)(ny + 1) * nx;
  const bool ok = face < nfaces;
  const long fc = ok ? face : 0;
  int ip, jp, iq, jq;
  if (DIR == 0) {  // x-face f of row j: nodes (f-1, j), (f, j)
    const int j = (int)(fc / (nx + 1)), f = (int)(fc - (long)j * (nx + 1));
    ip = f - 1; iq = f; jp = jq = j;
  } else {  // y-face gf of column i: nodes (i, gf-1), (i, gf)
    const int gf = (int)(fc / nx), i = (int)(fc - (long)gf * nx);
    ip = iq = i; jp = gf - 1; jq = gf;
  }
  double sum = 0.0;
  for (int b = 0; b < a.B; b++) {
    if (b * L + l >= a.N) continue;  // padding slices
    const double ap = true_value<DIR>(a, b, ip, jp, l), aq = true_value<DIR>(a, b, iq, jq, l);
    const double wp = true_value<DIR>(w, b, ip, jp, l), wq = true_value<DIR>(w, b, iq, jq, l);
    sum = fma(aq - ap, wq - wp, sum);
  }
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  if (ok && l == 0) g[face] += -coef * sum;
}

// out[s] = transpose of in[s] for count states of ny x nx (out is nx x ny).
__global__ void k_transpose_states(const double* __restrict__ in, double* __restrict__ out,
                                   int nx, int ny, int count) {
  __shared__ double t[32][33];
  const int s = blockIdx.z;
  if (s >= count) return;
  const long np = (long)nx * ny;
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + tx, j = j0 + r;
    t[r][tx] = (i < nx && j < ny) ? in[s * np + (long)j * nx + i] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j = j0 + tx, i = i0 + r;  // out[i][j]
    if (i < nx && j < ny) out[s * np + (long)i * ny + j] = t[tx][r];
  }
}

// out = true value of slice `slice` of an interleaved workspace after an x sweep.
__global__ void k_slice_xcorr(const DimInst* __restrict__ A, int slice, double* __restrict__ out) {
  const DimInst& a = A[0];
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)a.nx * a.ny) return;
  const int j = (int)(t / a.nx), i = (int)(t - (long)j * a.nx);
  out[t] = true_value<0>(a, slice / a.L, i, j, slice % a.L);
}

}  // namespace

hipError_t launch_face_grad_x(const double* nu, const double* W, int nx, int ny, double coef,
                              double* gax, hipStream_t s) {
  long total = (long)ny * (nx + 1);
  hipLaunchKernelGGL(k_face_grad_x, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, nu, W,
                     nx, ny, coef, gax);
  return hipGetLastError();
}

hipError_t launch_face_grad_y(const double* mu, const double* V, int nx, int ny, double coef,
                              double* gay, hipStream_t s) {
  long total = (long)(ny + 1) * nx;
  hipLaunchKernelGGL(k_face_grad_y, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, mu, V,
                     nx, ny, coef, gay);
  return hipGetLastError();
}

template <int DIR>
static hipError_t grad_faces_d(const DimInst* A, const DimInst* Bst, const DimInst& h, double coef,
                               double* g, hipStream_t s) {
  const long nfaces = DIR == 0 ? (long)h.ny * (h.nx + 1) : (long)(h.ny + 1) * h.nx;
  switch (h.L) {
#define PR_GF(LL)                                                                          \
  case LL:                                                                                 \
    hipLaunchKernelGGL((k_grad_faces<DIR, LL>), dim3((unsigned)((nfaces + 64 / LL - 1) / (64 / LL))), \
                       dim3(64), 0, s, A, Bst, coef, g);                                   \
    return hipGetLastError();
    PR_GF(8) PR_GF(16) PR_GF(32) PR_GF(64)
#undef PR_GF
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_grad_faces(int dir, const DimInst* A, const DimInst* Bst, const DimInst& h,
                             double coef, double* g, hipStream_t s) {
  return dir == 0 ? grad_faces_d<0>(A, Bst, h, coef, g, s) : grad_faces_d<1>(A, Bst, h, coef, g, s);
}

hipError_t launch_transpose_states(const double* in, double* out, int nx, int ny, int count,
                                   hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_states, dim3((nx + 31) / 32, (ny + 31) / 32, count), dim3(256), 0,
                     s, in, out, nx, ny, count);
  return hipGetLastError();
}

hipError_t launch_slice_xcorr(const DimInst* A, const DimInst& h, int slice, double* out,
                              hipStream_t s) {
  const long n = (long)h.nx * h.ny;
  hipLaunchKernelGGL(k_slice_xcorr, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, slice,
                     out);
  return hipGetLastError();
}

hipError_t launch_theta_chain(const double* theta, const double* gax, const double* gay, int nx,
                              int ny, double* gth, hipStream_t s) {
  long total = (long)(nx + 2) * (ny + 2);
  hipLaunchKernelGGL(k_theta_chain, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, theta,
                     gax, gay, nx, ny, gth);
  return hipGetLastError();
}

}  // namespace prk
