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

hipError_t launch_theta_chain(const double* theta, const double* gax, const double* gay, int nx,
                              int ny, double* gth, hipStream_t s) {
  long total = (long)(nx + 2) * (ny + 2);
  hipLaunchKernelGGL(k_theta_chain, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, theta,
                     gax, gay, nx, ny, gth);
  return hipGetLastError();
}

}  // namespace prk
