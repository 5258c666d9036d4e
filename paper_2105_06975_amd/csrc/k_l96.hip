// Lorenz-96 tangent linear (M_i) and adjoint (M_i^T) products, §7.1.
//
//   dx_j/dt = (x_{j+1} - x_{j-2}) x_{j-1} - x_j + F   (periodic in j)
// M_i is the Jacobian of nsteps classical RK4 steps of length dt started from the stored
// linearisation state x_{i-1}.  With J(y) d = (d_{j+1} - d_{j-2}) y_{j-1}
// + (y_{j+1} - y_{j-2}) d_{j-1} - d_j, one tangent step is
//   d1 = J(y1) a1, a1 = d;  d2 = J(y2)(d + h/2 d1);  d3 = J(y3)(d + h/2 d2);
//   d4 = J(y4)(d + h d3);   d' = d + h/6 (d1 + 2 d2 + 2 d3 + d4)
// with y1..y4 the nonlinear stage states.  The adjoint runs the same chain backwards with
//   (J(y)^T l)_m = y_{m-2} l_{m-1} - y_{m+1} l_{m+2} + (y_{m+2} - y_{m-1}) l_{m+1} - l_m,
// recomputing the stage states of each step from x_{i-1}.
// One workgroup per block product; the state (s <= 2048) lives in LDS.
#include "svar_impl.h"

namespace svar {

static constexpr int NT = 256;
static constexpr int MAXS = 2048;
static constexpr int EPT = MAXS / NT;

__device__ __forceinline__ int wrap(int j, int s) {
  j %= s;
  return j < 0 ? j + s : j;
}

// f(y)_j from an LDS copy of y
__device__ __forceinline__ double l96_f(const double* y, int j, int s, double F) {
  return (y[wrap(j + 1, s)] - y[wrap(j - 2, s)]) * y[wrap(j - 1, s)] - y[j] + F;
}
__device__ __forceinline__ double l96_jv(const double* y, const double* d, int j, int s) {
  return (d[wrap(j + 1, s)] - d[wrap(j - 2, s)]) * y[wrap(j - 1, s)] +
         (y[wrap(j + 1, s)] - y[wrap(j - 2, s)]) * d[wrap(j - 1, s)] - d[j];
}
__device__ __forceinline__ double l96_jtv(const double* y, const double* l, int m, int s) {
  return y[wrap(m - 2, s)] * l[wrap(m - 1, s)] - y[wrap(m + 1, s)] * l[wrap(m + 2, s)] +
         (y[wrap(m + 2, s)] - y[wrap(m - 1, s)]) * l[wrap(m + 1, s)] - l[m];
}

// one nonlinear RK4 step on registers x[] (elements j = tid + q NT), stage states written to
// Ys[0..3] (LDS) when Ys != nullptr; scratch ys is an LDS array of s doubles
__device__ void rk4_step(double* x, int s, double F, double h, double* ys, double* Ys) {
  double ks[EPT], k[EPT];
  // stage 1
  __syncthreads();
  for (int q = 0; q < EPT; ++q) {
    const int j = threadIdx.x + q * NT;
    if (j < s) {
      ys[j] = x[q];
      if (Ys) Ys[j] = x[q];
    }
  }
  __syncthreads();
  for (int q = 0; q < EPT; ++q) {
    const int j = threadIdx.x + q * NT;
    if (j < s) {
      k[q] = l96_f(ys, j, s, F);
      ks[q] = k[q];
    }
  }
  const double c[3] = {0.5 * h, 0.5 * h, h};
  const double wgt[3] = {2.0, 2.0, 1.0};
  for (int st = 0; st < 3; ++st) {
    __syncthreads();
    for (int q = 0; q < EPT; ++q) {
      const int j = threadIdx.x + q * NT;
      if (j < s) {
        const double v = x[q] + c[st] * k[q];
        ys[j] = v;
        if (Ys) Ys[(st + 1) * s + j] = v;
      }
    }
    __syncthreads();
    for (int q = 0; q < EPT; ++q) {
      const int j = threadIdx.x + q * NT;
      if (j < s) {
        k[q] = l96_f(ys, j, s, F);
        ks[q] += wgt[st] * k[q];
      }
    }
  }
  for (int q = 0; q < EPT; ++q) {
    const int j = threadIdx.x + q * NT;
    if (j < s) x[q] += h / 6.0 * ks[q];
  }
}

__global__ __launch_bounds__(NT) void k_mstep_l96(const MJob* __restrict__ jobs,
                                                  const ModelDev* __restrict__ models, Bases b,
                                                  const int* __restrict__ skip, int njobs) {
  if (skip && *skip) return;
  const int jid = blockIdx.y + 65535 * blockIdx.z;
  if (jid >= njobs || blockIdx.x != 0) return;
  extern __shared__ double lds[];
  const MJob J = jobs[jid];
  if (SVAR_JOB_SKIPPED(b, J)) return;
  const int s = J.s;
  const double* in = b.p[J.in.base] + J.in.off;
  double* out = b.p[J.out.base] + J.out.off;
  if (J.model < 0) {
    for (int j = threadIdx.x; j < s; j += NT) out[j] = in[j];
    return;
  }
  const ModelDev& M = models[J.model];
  const double F = M.F, h = M.dt;
  const int ns = M.nsteps;
  const double* x0 = M.traj + (size_t)(J.mi - 1) * s;
  const double* xin = b.p[J.x.base] + J.x.off;
  double* ys = lds;           // s
  double* as = lds + s;       // s
  double* Ys = lds + 2 * s;   // 4 s (adjoint only)
  double x[EPT], d[EPT];
  for (int q = 0; q < EPT; ++q) {
    const int j = threadIdx.x + q * NT;
    x[q] = j < s ? x0[j] : 0.0;
    d[q] = j < s ? xin[j] : 0.0;
  }
  if (!J.trans) {
    for (int n = 0; n < ns; ++n) {
      double k[EPT], dk[EPT], ks[EPT], dks[EPT];
      const double c[4] = {0.0, 0.5 * h, 0.5 * h, h};
      const double wgt[4] = {1.0, 2.0, 2.0, 1.0};
      for (int q = 0; q < EPT; ++q) {
        k[q] = 0.0;
        dk[q] = 0.0;
        ks[q] = 0.0;
        dks[q] = 0.0;
      }
      for (int st = 0; st < 4; ++st) {
        __syncthreads();
        for (int q = 0; q < EPT; ++q) {
          const int j = threadIdx.x + q * NT;
          if (j < s) {
            ys[j] = x[q] + c[st] * k[q];
            as[j] = d[q] + c[st] * dk[q];
          }
        }
        __syncthreads();
        for (int q = 0; q < EPT; ++q) {
          const int j = threadIdx.x + q * NT;
          if (j < s) {
            k[q] = l96_f(ys, j, s, F);
            dk[q] = l96_jv(ys, as, j, s);
            ks[q] += wgt[st] * k[q];
            dks[q] += wgt[st] * dk[q];
          }
        }
      }
      for (int q = 0; q < EPT; ++q) {
        x[q] += h / 6.0 * ks[q];
        d[q] += h / 6.0 * dks[q];
      }
    }
  } else {
    // reverse over the steps; the stage states of step n are recomputed from x_{i-1}
    for (int n = ns - 1; n >= 0; --n) {
      double xs[EPT];
      for (int q = 0; q < EPT; ++q) xs[q] = x[q];
      for (int m = 0; m < n; ++m) rk4_step(xs, s, F, h, ys, nullptr);
      rk4_step(xs, s, F, h, ys, Ys);  // Ys[0..3] = stage states of step n
      double lam[EPT], ld[4][EPT];
      const double wl[4] = {h / 6.0, h / 3.0, h / 3.0, h / 6.0};
      for (int q = 0; q < EPT; ++q) {
        lam[q] = d[q];
        for (int st = 0; st < 4; ++st) ld[st][q] = wl[st] * d[q];
      }
      const double back[4] = {0.0, 0.5 * h, 0.5 * h, h};  // a_st = d + back[st] d_{st-1}
      for (int st = 3; st >= 0; --st) {
        __syncthreads();
        for (int q = 0; q < EPT; ++q) {
          const int j = threadIdx.x + q * NT;
          if (j < s) as[j] = ld[st][q];
        }
        __syncthreads();
        for (int q = 0; q < EPT; ++q) {
          const int j = threadIdx.x + q * NT;
          if (j < s) {
            const double la = l96_jtv(Ys + st * s, as, j, s);
            lam[q] += la;
            if (st > 0) ld[st - 1][q] += back[st] * la;
          }
        }
      }
      for (int q = 0; q < EPT; ++q) d[q] = lam[q];
    }
  }
  __syncthreads();
  for (int q = 0; q < EPT; ++q) {
    const int j = threadIdx.x + q * NT;
    if (j < s) out[j] = in[j] + J.alpha * d[q];
  }
}

// y_0 = x_0, y_i = nonlinear model over one observation interval from x_{i-1} (i = 1..N);
// one workgroup per block, the state in registers and an LDS copy for the neighbours.
__global__ __launch_bounds__(NT) void k_l96_forecast(const double* __restrict__ x,
                                                     double* __restrict__ y, int s, int N, double F,
                                                     double h, int nsteps) {
  __shared__ double ys[MAXS];
  const int i = blockIdx.x;
  if (i > N) return;
  double xr[EPT];
  for (int q = 0; q < EPT; ++q) {
    const int j = threadIdx.x + q * NT;
    xr[q] = j < s ? x[(size_t)(i > 0 ? i - 1 : 0) * s + j] : 0.0;
  }
  if (i > 0)
    for (int n = 0; n < nsteps; ++n) rk4_step(xr, s, F, h, ys, nullptr);
  for (int q = 0; q < EPT; ++q) {
    const int j = threadIdx.x + q * NT;
    if (j < s) y[(size_t)i * s + j] = xr[q];
  }
}

void launch_l96_forecast(const double* x, double* y, int s, int N, double F, double h, int nsteps,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_l96_forecast, dim3(N + 1), dim3(NT), 0, st, x, y, s, N, F, h, nsteps);
}

void launch_mstep_l96(const MJob* jobs, int njobs, int max_s, const ModelDev* models, Bases b,
                      const int* skip, hipStream_t st) {
  if (njobs == 0) return;
  (void)max_s;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_mstep_l96, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(6 * MAXS * sizeof(double)));
    attr = true;
  }
  const dim3 grid = njobs <= 65535 ? dim3(1, njobs, 1) : dim3(1, 65535, (njobs + 65534) / 65535);
  hipLaunchKernelGGL(k_mstep_l96, grid, dim3(NT), (size_t)6 * MAXS * sizeof(double), st, jobs,
                     models, b, skip, njobs);
}

}  // namespace svar
