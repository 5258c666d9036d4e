// Set-up kernels: everything the preconditioners need before the iteration (§6.2: Rhat_i is
// precomputed and stored), built on the GPU.
//
//  * Explicit SPD inverses (Rhat_i^{-1}, Dhat_i^{-1}) by the Newton-Schulz iteration
//    X <- X (2I - A X) started from X0 = I / ||A||_inf; its products run on the MFMA GEMM.
//  * Extreme eigenpairs of R_i (gamma = lambda_min for ridge regression, the two smallest
//    eigenpairs for the minimum-eigenvalue method, §6.1) by repeated squaring of the
//    normalised inverse, which converges to the projector on the smallest eigenvector.
//  * Taps of the periodic tridiagonal inverse T^{-1} (implicit advection-diffusion step).
//  * Float32 / bfloat16 copies of covariance matrices for the mixed-precision paths.
#include "svar_impl.h"
#include "setup.h"

namespace svar {

static constexpr int NT = 256;

static unsigned gsz(int64_t n, int cap = 8192) {
  int64_t g = (n + NT - 1) / NT;
  if (g < 1) g = 1;
  return (unsigned)(g > cap ? cap : g);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ double bsum(double v) {
  __shared__ double red[NT / 64];
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < NT / 64; ++i) t += red[i];
  return t;
}

#define GRID_LOOP(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < (n); i += (int64_t)gridDim.x * NT)

__global__ __launch_bounds__(NT) void k_scaled_identity(double* X, int n, double a) {
  GRID_LOOP(e, (int64_t)n * n) {
    const int64_t r = e / n, c = e - r * n;
    X[e] = r == c ? a : 0.0;
  }
}

// part[block] = sum over this block's elements of (I - T)^2; then T <- 2I - T
__global__ __launch_bounds__(NT) void k_ns_residual(double* T, int n, double* part) {
  double acc = 0.0;
  GRID_LOOP(e, (int64_t)n * n) {
    const int64_t r = e / n, c = e - r * n;
    const double id = r == c ? 1.0 : 0.0;
    const double d = id - T[e];
    acc += d * d;
    T[e] = id + d;
  }
  acc = bsum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(NT) void k_rowabs(const double* A, int n, double* out) {
  const int r = blockIdx.x;
  double acc = 0.0;
  for (int c = threadIdx.x; c < n; c += NT) acc += fabs(A[(int64_t)r * n + c]);
  acc = bsum(acc);
  if (threadIdx.x == 0) out[r] = acc;
}

__global__ __launch_bounds__(NT) void k_symmetrize(double* X, int n) {
  GRID_LOOP(e, (int64_t)n * n) {
    const int64_t r = e / n, c = e - r * n;
    if (r < c) {
      const double m = 0.5 * (X[r * n + c] + X[c * n + r]);
      X[r * n + c] = m;
      X[c * n + r] = m;
    }
  }
}

__global__ __launch_bounds__(NT) void k_copy_scale_shift(const double* A, double* X, int n,
                                                         double a, double d) {
  GRID_LOOP(e, (int64_t)n * n) {
    const int64_t r = e / n, c = e - r * n;
    X[e] = a * A[e] + (r == c ? d : 0.0);
  }
}

__global__ __launch_bounds__(NT) void k_scale_inplace(double* X, int64_t len, double a) {
  GRID_LOOP(e, len) X[e] *= a;
}

__global__ __launch_bounds__(NT) void k_sqdiff_part(const double* X, const double* Y, int64_t len,
                                                    double* part) {
  double acc = 0.0;
  GRID_LOOP(e, len) {
    const double d = X[e] - (Y ? Y[e] : 0.0);
    acc += d * d;
  }
  acc = bsum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(NT) void k_dot_part(const double* a, const double* b, int64_t len,
                                                 double* part) {
  double acc = 0.0;
  GRID_LOOP(e, len) acc += a[e] * b[e];
  acc = bsum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// squared norm of every row of a (symmetric) matrix
__global__ __launch_bounds__(NT) void k_rownorm2(const double* M, int n, double* out) {
  const int r = blockIdx.x;
  double acc = 0.0;
  for (int c = threadIdx.x; c < n; c += NT) {
    const double v = M[(int64_t)r * n + c];
    acc += v * v;
  }
  acc = bsum(acc);
  if (threadIdx.x == 0) out[r] = acc;
}

__global__ __launch_bounds__(NT) void k_row_scaled(const double* M, int n, int row, double a,
                                                   double* v) {
  GRID_LOOP(c, n) v[c] = a * M[(int64_t)row * n + c];
}

__global__ __launch_bounds__(NT) void k_rank1(double* X, int n, const double* v, double c) {
  GRID_LOOP(e, (int64_t)n * n) {
    const int64_t r = e / n, q = e - r * n;
    X[e] += c * v[r] * v[q];
  }
}

__global__ __launch_bounds__(NT) void k_diag_inv(const double* R, int n, double* out) {
  GRID_LOOP(i, n) out[i] = 1.0 / R[i * (int64_t)n + i];
}

// First column g of T^{-1} for the periodic tridiagonal (T x)_j = a x_{j-1} + b x_j + c x_{j+1}.
// T = T' + u v^T with u = (gam, 0, .., 0, c), v = (1, 0, .., 0, a / gam), gam = -b, T'
// tridiagonal; x = y - (v^T y / (1 + v^T z)) z with T' y = e_0, T' z = u (Sherman-Morrison).
// One thread: a set-up step of O(s) work.  work holds 3 s doubles.
__global__ void k_tridiag_inv_col(double a, double b, double c, int s, double* g, double* work) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double* cp = work;
  double* y = work + s;
  double* z = work + 2 * s;
  const double gam = -b;
  // forward elimination for both right-hand sides
  double d0 = b - gam;
  cp[0] = c / d0;
  y[0] = 1.0 / d0;
  z[0] = gam / d0;
  for (int j = 1; j < s; ++j) {
    const double dj = (j == s - 1) ? b - c * a / gam : b;
    const double m = dj - a * cp[j - 1];
    cp[j] = (j < s - 1) ? c / m : 0.0;
    const double rj = 0.0;
    const double uj = (j == s - 1) ? c : 0.0;
    y[j] = (rj - a * y[j - 1]) / m;
    z[j] = (uj - a * z[j - 1]) / m;
  }
  for (int j = s - 2; j >= 0; --j) {
    y[j] -= cp[j] * y[j + 1];
    z[j] -= cp[j] * z[j + 1];
  }
  const double vy = y[0] + (a / gam) * y[s - 1];
  const double vz = z[0] + (a / gam) * z[s - 1];
  const double f = vy / (1.0 + vz);
  for (int j = 0; j < s; ++j) g[j] = y[j] - f * z[j];
}

__device__ __forceinline__ unsigned short f2bf_rne(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__global__ __launch_bounds__(NT) void k_to_f32(const double* src, float* dst, int64_t len) {
  GRID_LOOP(e, len) dst[e] = (float)src[e];
}
// dst[r ld + c] = src[r n + c] for c < n, 0 for n <= c < ld
__global__ __launch_bounds__(NT) void k_to_f32_pad(const double* src, float* dst, int n, int ld) {
  const int64_t len = (int64_t)n * ld;
  GRID_LOOP(e, len) {
    const int64_t r = e / ld;
    const int c = (int)(e - r * ld);
    dst[e] = c < n ? (float)src[r * n + c] : 0.0f;
  }
}
__global__ __launch_bounds__(NT) void k_to_bf16(const double* src, unsigned short* dst, int64_t len) {
  GRID_LOOP(e, len) dst[e] = f2bf_rne((float)src[e]);
}

// ------------------------------------------------------------------ launchers
// out[j] = ||R[pst_j..pst_{j+1}), pst_{j+1}..pst_{j+2})||_F / sqrt(pvec_j pvec_{j+1}) for the
// super-diagonal blocks of R (n x n row-major), one workgroup per block pair
__global__ __launch_bounds__(NT) void k_superdiag_norms(const double* R, int n,
                                                        const int* pst, double* out) {
  __shared__ double red[NT / 64];
  const int j = blockIdx.x;
  const int r0 = pst[j], r1 = pst[j + 1], c1 = pst[j + 2];
  const int rows = r1 - r0, cols = c1 - r1;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)rows * cols; e += NT) {
    const int r = (int)(e / cols), c = (int)(e - (int64_t)r * cols);
    const double v = R[(int64_t)(r0 + r) * n + r1 + c];
    acc += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    out[j] = sqrt(t) / sqrt((double)rows * (double)cols);
  }
}

void su_superdiag_norms(const double* R, int n, const int* pst, int npairs, double* out,
                        hipStream_t st) {
  if (npairs > 0)
    hipLaunchKernelGGL(k_superdiag_norms, dim3(npairs), dim3(NT), 0, st, R, n, pst, out);
}

void su_scaled_identity(double* X, int n, double a, hipStream_t st) {
  hipLaunchKernelGGL(k_scaled_identity, dim3(gsz((int64_t)n * n)), dim3(NT), 0, st, X, n, a);
}
int su_ns_residual(double* T, int n, double* part, hipStream_t st) {
  const unsigned g = gsz((int64_t)n * n, 1024);
  hipLaunchKernelGGL(k_ns_residual, dim3(g), dim3(NT), 0, st, T, n, part);
  return (int)g;
}
void su_rowabs(const double* A, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_rowabs, dim3(n), dim3(NT), 0, st, A, n, out);
}
void su_symmetrize(double* X, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_symmetrize, dim3(gsz((int64_t)n * n)), dim3(NT), 0, st, X, n);
}
void su_copy_scale_shift(const double* A, double* X, int n, double a, double d, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_scale_shift, dim3(gsz((int64_t)n * n)), dim3(NT), 0, st, A, X, n, a, d);
}
void su_scale(double* X, int64_t len, double a, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_inplace, dim3(gsz(len)), dim3(NT), 0, st, X, len, a);
}
int su_sqdiff_part(const double* X, const double* Y, int64_t len, double* part, hipStream_t st) {
  const unsigned g = gsz(len, 1024);
  hipLaunchKernelGGL(k_sqdiff_part, dim3(g), dim3(NT), 0, st, X, Y, len, part);
  return (int)g;
}
int su_dot_part(const double* a, const double* b, int64_t len, double* part, hipStream_t st) {
  const unsigned g = gsz(len, 1024);
  hipLaunchKernelGGL(k_dot_part, dim3(g), dim3(NT), 0, st, a, b, len, part);
  return (int)g;
}
void su_rownorm2(const double* M, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_rownorm2, dim3(n), dim3(NT), 0, st, M, n, out);
}
void su_row_scaled(const double* M, int n, int row, double a, double* v, hipStream_t st) {
  hipLaunchKernelGGL(k_row_scaled, dim3(gsz(n)), dim3(NT), 0, st, M, n, row, a, v);
}
void su_rank1(double* X, int n, const double* v, double c, hipStream_t st) {
  hipLaunchKernelGGL(k_rank1, dim3(gsz((int64_t)n * n)), dim3(NT), 0, st, X, n, v, c);
}
void su_diag_inv(const double* R, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_inv, dim3(gsz(n)), dim3(NT), 0, st, R, n, out);
}
void su_tridiag_inv_col(double a, double b, double c, int s, double* g, double* work,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_tridiag_inv_col, dim3(1), dim3(64), 0, st, a, b, c, s, g, work);
}
void su_to_f32(const double* src, void* dst, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(k_to_f32, dim3(gsz(len)), dim3(NT), 0, st, src, (float*)dst, len);
}
void su_to_f32_pad(const double* src, void* dst, int n, int ld, hipStream_t st) {
  const int64_t len = (int64_t)n * ld;
  hipLaunchKernelGGL(k_to_f32_pad, dim3(gsz(len)), dim3(NT), 0, st, src, (float*)dst, n, ld);
}
void su_to_bf16(const double* src, void* dst, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3(gsz(len)), dim3(NT), 0, st, src, (unsigned short*)dst, len);
}

}  // namespace svar
