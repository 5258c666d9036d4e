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
#include "svar_impl.h"

namespace svar {

static constexpr int NT = 256;

__device__ __forceinline__ int wrap(int j, int s) {
  j %= s;
  return j < 0 ? j + s : j;
}

// Tiled products: a workgroup owns TILE outputs [j0, j0 + TILE) of one block product and works
// on a region of the ring that extends the tile by the dependence radius of the chain, so any s
// (and several workgroups per product) works.  f and J at point j read j-2 .. j+1, J^T at
// point m reads m-2 .. m+2.  Region indices i map to ring points (j0 - left + i) mod s; values
// near the region's edges become invalid stage by stage (their neighbours are missing) but
// never reach the tile, whose distance to the edges is the chain's radius:
//   tangent of ns steps: left 8 ns, right 4 ns;
//   adjoint: the cotangent needs 8 ns on both sides, and the nonlinear stage states it uses
//   are recomputed forward from x_{i-1} over that range plus 8 ns left, 4 ns right.
static constexpr int TILE = 256;
static constexpr int L96_MAX_STEPS = 32;  // region <= TILE + 28 * 32 points (LDS below)
static constexpr int REG_MAX = TILE + 28 * L96_MAX_STEPS + 8;
// LDS arrays of the adjoint, each of its region length: x, ys, k, ks, the 4 stage states Ys,
// lam, the 4 stage cotangents ld, as (ADJ_ARRAYS * REG_MAX doubles = 130 KB at 32 steps)
static constexpr int ADJ_ARRAYS = 14;

// stage value of f or J v at region index i from LDS copies (i - 2 .. i + 1 in range)
__device__ __forceinline__ double reg_f(const double* y, int i, double F) {
  return (y[i + 1] - y[i - 2]) * y[i - 1] - y[i] + F;
}
__device__ __forceinline__ double reg_jv(const double* y, const double* d, int i) {
  return (d[i + 1] - d[i - 2]) * y[i - 1] + (y[i + 1] - y[i - 2]) * d[i - 1] - d[i];
}
__device__ __forceinline__ double reg_jtv(const double* y, const double* l, int m) {
  return y[m - 2] * l[m - 1] - y[m + 1] * l[m + 2] + (y[m + 2] - y[m - 1]) * l[m + 1] - l[m];
}

// one nonlinear RK4 step over the region (x in place); stage states to Ys[0..3] when given
__device__ void reg_rk4(double* x, double* ys, double* k, double* ks, double* Ys, int R,
                        double F, double h) {
  const double c[4] = {0.0, 0.5 * h, 0.5 * h, h};
  const double wgt[4] = {1.0, 2.0, 2.0, 1.0};
  for (int st = 0; st < 4; ++st) {
    __syncthreads();
    for (int i = threadIdx.x; i < R; i += NT) {
      const double v = x[i] + (st ? c[st] * k[i] : 0.0);
      ys[i] = v;
      if (Ys) Ys[st * R + i] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < R; i += NT) {
      const double kv = (i >= 2 && i + 1 < R) ? reg_f(ys, i, F) : 0.0;
      k[i] = kv;
      ks[i] = (st ? ks[i] : 0.0) + wgt[st] * kv;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R; i += NT) x[i] += h / 6.0 * ks[i];
}

__global__ __launch_bounds__(NT) void k_mstep_l96(const MJob* __restrict__ jobs,
                                                  const ModelDev* __restrict__ models, Bases b,
                                                  const int* __restrict__ skip, int njobs) {
  if (skip && *skip) return;
  const int jid = blockIdx.y + 65535 * blockIdx.z;
  if (jid >= njobs) return;
  extern __shared__ double lds[];
  const MJob J = jobs[jid];
  if (SVAR_JOB_SKIPPED(b, J)) return;
  const int s = J.s;
  const int j0 = blockIdx.x * TILE;
  if (j0 >= s) return;
  const int tlen = min(TILE, s - j0);
  const double* in = b.p[J.in.base] + J.in.off;
  double* out = b.p[J.out.base] + J.out.off;
  if (J.model < 0) {
    for (int t = threadIdx.x; t < tlen; t += NT) out[j0 + t] = in[j0 + t];
    return;
  }
  const ModelDev& M = models[J.model];
  const double F = M.F, h = M.dt;
  const int ns = M.nsteps;
  const double* x0 = M.traj + (size_t)(J.mi - 1) * s;
  const double* xin = b.p[J.x.base] + J.x.off;
  if (!J.trans) {
    const int left = 8 * ns + 2, R = TILE + 12 * ns + 4;
    double* x = lds;          // nonlinear state
    double* d = x + R;        // tangent
    double* ys = d + R;
    double* as = ys + R;
    double* k = as + R;
    double* dk = k + R;
    double* ks = dk + R;
    double* dks = ks + R;
    for (int i = threadIdx.x; i < R; i += NT) {
      const int g = wrap(j0 - left + i, s);
      x[i] = x0[g];
      d[i] = xin[g];
    }
    const double c[4] = {0.0, 0.5 * h, 0.5 * h, h};
    const double wgt[4] = {1.0, 2.0, 2.0, 1.0};
    for (int n = 0; n < ns; ++n) {
      for (int st = 0; st < 4; ++st) {
        __syncthreads();
        for (int i = threadIdx.x; i < R; i += NT) {
          ys[i] = x[i] + (st ? c[st] * k[i] : 0.0);
          as[i] = d[i] + (st ? c[st] * dk[i] : 0.0);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < R; i += NT) {
          const bool ok = i >= 2 && i + 1 < R;
          const double kv = ok ? reg_f(ys, i, F) : 0.0;
          const double dv = ok ? reg_jv(ys, as, i) : 0.0;
          k[i] = kv;
          dk[i] = dv;
          ks[i] = (st ? ks[i] : 0.0) + wgt[st] * kv;
          dks[i] = (st ? dks[i] : 0.0) + wgt[st] * dv;
        }
      }
      __syncthreads();
      for (int i = threadIdx.x; i < R; i += NT) {
        x[i] += h / 6.0 * ks[i];
        d[i] += h / 6.0 * dks[i];
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < tlen; t += NT)
      out[j0 + t] = in[j0 + t] + J.alpha * d[left + t];
    return;
  }
  // adjoint: before step n (taken in reverse) the cotangent must be valid 8 (n + 1) points
  // around the tile and the stage states of step n 2 points further; stage 3 of step n is
  // valid from 8 n + 6 to R - 4 n - 3, so the tile starts at 16 ns + 4 and the region ends
  // 12 ns + 4 points after it (both with a little slack)
  const int left = 16 * ns + 4, R = TILE + 28 * ns + 8;
  double* x = lds;
  double* ys = x + R;
  double* k = ys + R;
  double* ks = k + R;
  double* Ys = ks + R;       // 4 R
  double* lam = Ys + 4 * R;  // cotangent after the current step (region indices)
  double* ld = lam + R;      // 4 R: stage cotangents
  double* as = ld + 4 * R;
  for (int i = threadIdx.x; i < R; i += NT) lam[i] = xin[wrap(j0 - left + i, s)];
  const double wl[4] = {h / 6.0, h / 3.0, h / 3.0, h / 6.0};
  const double back[4] = {0.0, 0.5 * h, 0.5 * h, h};
  for (int n = ns - 1; n >= 0; --n) {
    __syncthreads();
    for (int i = threadIdx.x; i < R; i += NT) x[i] = x0[wrap(j0 - left + i, s)];
    for (int m = 0; m < n; ++m) reg_rk4(x, ys, k, ks, nullptr, R, F, h);
    reg_rk4(x, ys, k, ks, Ys, R, F, h);  // Ys[0..3]: stage states of step n
    __syncthreads();
    for (int i = threadIdx.x; i < R; i += NT)
      for (int st = 0; st < 4; ++st) ld[st * R + i] = wl[st] * lam[i];
    for (int st = 3; st >= 0; --st) {
      __syncthreads();
      for (int i = threadIdx.x; i < R; i += NT) as[i] = ld[st * R + i];
      __syncthreads();
      for (int i = threadIdx.x; i < R; i += NT) {
        const double la = (i >= 2 && i + 2 < R) ? reg_jtv(Ys + st * R, as, i) : 0.0;
        lam[i] += la;
        if (st > 0) ld[(st - 1) * R + i] += back[st] * la;
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < tlen; t += NT)
    out[j0 + t] = in[j0 + t] + J.alpha * lam[left + t];
}

// y_0 = x_0, y_i = nonlinear model over one observation interval from x_{i-1} (i = 1..N); a
// workgroup per (tile, block), the region extended by 8 ns left and 4 ns right.
__global__ __launch_bounds__(NT) void k_l96_forecast(const double* __restrict__ x,
                                                     double* __restrict__ y, int s, int N, double F,
                                                     double h, int nsteps) {
  extern __shared__ double lds[];
  const int i = blockIdx.y;
  const int j0 = blockIdx.x * TILE;
  if (i > N || j0 >= s) return;
  const int tlen = min(TILE, s - j0);
  if (i == 0) {
    for (int t = threadIdx.x; t < tlen; t += NT) y[j0 + t] = x[j0 + t];
    return;
  }
  const int left = 8 * nsteps + 2, R = TILE + 12 * nsteps + 4;
  double* xr = lds;
  double* ys = xr + R;
  double* k = ys + R;
  double* ks = k + R;
  const double* xp = x + (size_t)(i - 1) * s;
  for (int q = threadIdx.x; q < R; q += NT) xr[q] = xp[wrap(j0 - left + q, s)];
  for (int n = 0; n < nsteps; ++n) reg_rk4(xr, ys, k, ks, nullptr, R, F, h);
  __syncthreads();
  for (int t = threadIdx.x; t < tlen; t += NT) y[(size_t)i * s + j0 + t] = xr[left + t];
}

void launch_l96_forecast(const double* x, double* y, int s, int N, double F, double h, int nsteps,
                         hipStream_t st) {
  const size_t sh = (size_t)4 * (TILE + 12 * nsteps + 4) * sizeof(double);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_l96_forecast,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(4 * (TILE + 12 * L96_MAX_STEPS + 4) * sizeof(double)));
    attr = true;
  }
  hipLaunchKernelGGL(k_l96_forecast, dim3((s + TILE - 1) / TILE, N + 1), dim3(NT), sh, st, x, y,
                     s, N, F, h, nsteps);
}

void launch_mstep_l96(const MJob* jobs, int njobs, int max_s, int max_steps,
                      const ModelDev* models, Bases b, const int* skip, hipStream_t st) {
  if (njobs == 0) return;
  // LDS for the largest step count of the launch's models (the adjoint's ADJ_ARRAYS arrays of
  // TILE + 28 ns + 8 points; the tangent needs 8 of TILE + 12 ns + 4)
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_mstep_l96, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(ADJ_ARRAYS * REG_MAX * sizeof(double)));
    attr = true;
  }
  const int ns = max_steps < 1 ? 1 : (max_steps > L96_MAX_STEPS ? L96_MAX_STEPS : max_steps);
  const size_t sh = (size_t)ADJ_ARRAYS * (TILE + 28 * ns + 8) * sizeof(double);
  const unsigned gx = (unsigned)((max_s + TILE - 1) / TILE);
  const dim3 grid = njobs <= 65535 ? dim3(gx, njobs, 1) : dim3(gx, 65535, (njobs + 65534) / 65535);
  hipLaunchKernelGGL(k_mstep_l96, grid, dim3(NT), sh, st, jobs, models, b, skip, njobs);
}

}  // namespace svar
