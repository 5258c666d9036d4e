// Preconditioned MINRES on the device (§3, §7: block-diagonal P_D is symmetric positive
// definite, so MINRES applies).  Lanczos in the P^{-1} inner product with the three-term
// recurrence; the tridiagonal least-squares problem is updated by one Givens rotation per
// step; x is updated with the last two search directions.  Many systems run in lock step,
// each with its own scalars.  Stopping test (§7: a residual criterion in the two norm): the
// residual r = rhs - A x is carried along with x.  Since x_k = x_{k-1} + phi_k w_k and
// w_k = (v_k - eps w_{k-2} - delta w_{k-1}) / gamma, A w_k follows the same recurrence from the
// product A v_k that the Lanczos step forms anyway, and r_k = r_{k-1} - phi_k A w_k; the
// iteration stops when ||r_k||_2 <= rtol ||rhs||_2.  Optionally the Paige-Saunders estimate of
// the P^{-1}-norm residual (phibar <= rtol * beta_1) is the test instead.
#include <algorithm>
#include <cmath>
#include <limits>

#include "mem.h"
#include "minres.h"

namespace svar {

static constexpr int NT = 256;

struct MState {
  int32_t done, iters, status, pad;  // pad: the step just taken met the stopping test
  double beta, beta_old, beta1, phibar, c, s, dbar, eps;
  double alpha, eps_old, delta, gamma, phi, tol;
  double tol2;   // rtol ||rhs||_2 (two-norm test)
  double res2;   // ||r_k||_2 of the carried residual
};

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

// part[task] = a . b over the task's range
__global__ __launch_bounds__(NT) void k_mr_dot(const KTask* __restrict__ tasks,
                                               const double* __restrict__ a,
                                               const double* __restrict__ b,
                                               double* __restrict__ part) {
  const KTask t = tasks[blockIdx.x];
  double acc = 0.0;
  for (int64_t e = t.e0 + threadIdx.x; e < t.e1; e += NT) acc += a[e] * b[e];
  acc = bsum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// beta_1 = sqrt(r^T P^{-1} r) from sysv; initial QR state
__global__ void k_mr_init(MState* __restrict__ st, const double* __restrict__ sysv,
                          const double* __restrict__ rhs2, double rtol, int nsys,
                          KGlobal* __restrict__ gl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int rem = 0;
  for (int i = 0; i < nsys; ++i) {
    MState S{};
    const double b2 = sysv[i];
    S.beta1 = b2 > 0.0 ? sqrt(b2) : 0.0;
    S.beta = S.beta1;
    S.phibar = S.beta1;
    S.c = -1.0;
    S.s = 0.0;
    S.tol = rtol * S.beta1;
    S.res2 = sqrt(fmax(rhs2[i], 0.0));
    S.tol2 = rtol * S.res2;
    S.done = (S.beta1 > 0.0) ? 0 : 1;
    if (!isfinite(b2) || b2 < 0.0) {
      S.done = 1;
      S.status = SVAR_E_BREAKDOWN;
    }
    st[i] = S;
    rem += S.done ? 0 : 1;
  }
  gl->j = 0;
  gl->remaining = rem;
  gl->all_done = rem == 0;
}

// v = y / beta
__global__ __launch_bounds__(NT) void k_mr_v(const KTask* __restrict__ tasks,
                                             const MState* __restrict__ st,
                                             const KGlobal* __restrict__ gl,
                                             const double* __restrict__ y, double* __restrict__ v) {
  if (gl->all_done) return;
  const KTask t = tasks[blockIdx.x];
  const MState S = st[t.sys];
  if (S.done) return;
  const double ib = 1.0 / S.beta;
  for (int64_t e = t.e0 + threadIdx.x; e < t.e1; e += NT) v[e] = y[e] * ib;
}

// y -= (beta / beta_old) r_prev (from the second step on); part = v . y
__global__ __launch_bounds__(NT) void k_mr_y1(const KTask* __restrict__ tasks,
                                              const MState* __restrict__ st,
                                              const KGlobal* __restrict__ gl, double* __restrict__ y,
                                              const double* __restrict__ rp,
                                              const double* __restrict__ v, int first,
                                              double* __restrict__ part,
                                              double* __restrict__ av) {
  if (gl->all_done) return;
  const KTask t = tasks[blockIdx.x];
  const MState S = st[t.sys];
  if (S.done) return;
  const double f = first ? 0.0 : S.beta / S.beta_old;
  double acc = 0.0;
  for (int64_t e = t.e0 + threadIdx.x; e < t.e1; e += NT) {
    double yy = y[e];
    if (av) av[e] = yy;  // A v, kept for the residual recurrence
    if (!first) yy -= f * rp[e];
    y[e] = yy;
    acc += v[e] * yy;
  }
  acc = bsum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// alpha = sysv; y -= (alpha / beta) r
__global__ __launch_bounds__(NT) void k_mr_y2(const KTask* __restrict__ tasks,
                                              const KSys* __restrict__ sys,
                                              MState* __restrict__ st,
                                              const KGlobal* __restrict__ gl,
                                              const double* __restrict__ sysv,
                                              double* __restrict__ y, const double* __restrict__ r) {
  if (gl->all_done) return;
  const KTask t = tasks[blockIdx.x];
  const MState S = st[t.sys];
  if (S.done) return;
  const double alpha = sysv[t.sys];
  const double f = alpha / S.beta;
  for (int64_t e = t.e0 + threadIdx.x; e < t.e1; e += NT) y[e] -= f * r[e];
  if (threadIdx.x == 0 && blockIdx.x == (unsigned)sys[t.sys].task0) st[t.sys].alpha = alpha;
}

// new beta from sysv = r^T P^{-1} r; Givens update of the tridiagonal QR
__global__ void k_mr_scalar(MState* __restrict__ st, const double* __restrict__ sysv, int nsys,
                            KGlobal* __restrict__ gl, int pnorm, double* __restrict__ hist,
                            int hlen) {
  if (gl->all_done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsys) return;
  MState S = st[i];
  if (S.done) return;
  const double b2 = sysv[i];
  const double beta = b2 > 0.0 ? sqrt(b2) : 0.0;
  S.beta_old = S.beta;
  S.eps_old = S.eps;
  S.delta = S.c * S.dbar + S.s * S.alpha;
  const double gbar = S.s * S.dbar - S.c * S.alpha;
  S.eps = S.s * beta;
  S.dbar = -S.c * beta;
  double gam = hypot(gbar, beta);
  if (!(gam > 0.0)) gam = 1e-300;
  S.gamma = gam;
  S.c = gbar / gam;
  S.s = beta / gam;
  S.phi = S.c * S.phibar;
  S.phibar = S.s * S.phibar;
  S.beta = beta;
  S.iters += 1;
  bool stop = false;
  if (!isfinite(S.phibar) || !isfinite(b2) || b2 < 0.0) {
    S.status = SVAR_E_BREAKDOWN;
    stop = true;
  } else if ((pnorm && S.phibar <= S.tol) || beta == 0.0) {
    stop = true;
  }
  // the x update of this step still runs (k_mr_w reads done only through `pending`)
  S.pad = stop ? 1 : 0;
  st[i] = S;
  if (hist && pnorm && S.iters <= hlen) hist[(int64_t)i * hlen + S.iters - 1] = S.phibar;
}

// two-norm test on the carried residual (sysv = ||r_k||^2 per system)
__global__ void k_mr_check(MState* __restrict__ st, const double* __restrict__ sysv, int nsys,
                           const KGlobal* __restrict__ gl, double* __restrict__ hist, int hlen) {
  if (gl->all_done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsys) return;
  MState S = st[i];
  if (S.done) return;
  const double r2 = sysv[i];
  S.res2 = r2 > 0.0 ? sqrt(r2) : 0.0;
  if (!isfinite(r2)) {
    S.status = SVAR_E_BREAKDOWN;
    S.pad = 1;
  } else if (S.res2 <= S.tol2) {
    S.pad = 1;
  }
  st[i] = S;
  if (hist && S.iters <= hlen) hist[(int64_t)i * hlen + S.iters - 1] = S.res2;
}

// w_new = (v - eps_old w_older - delta w_old) / gamma ; x += phi w_new; retire finished systems
__global__ __launch_bounds__(NT) void k_mr_w(const KTask* __restrict__ tasks,
                                             const KSys* __restrict__ sys,
                                             MState* __restrict__ st, KGlobal* __restrict__ gl,
                                             const double* __restrict__ v,
                                             const double* __restrict__ wolder,
                                             const double* __restrict__ wold,
                                             double* __restrict__ wnew, double* __restrict__ x,
                                             int first, const double* __restrict__ av,
                                             const double* __restrict__ awolder,
                                             const double* __restrict__ awold,
                                             double* __restrict__ awnew, double* __restrict__ res,
                                             double* __restrict__ part) {
  if (gl->all_done) return;
  const KTask t = tasks[blockIdx.x];
  const MState S = st[t.sys];
  if (S.done) return;
  const double ig = 1.0 / S.gamma;
  double acc = 0.0;
  for (int64_t e = t.e0 + threadIdx.x; e < t.e1; e += NT) {
    const double a = first ? 0.0 : wolder[e];
    const double b = first ? 0.0 : wold[e];
    const double wn = (v[e] - S.eps_old * a - S.delta * b) * ig;
    wnew[e] = wn;
    x[e] += S.phi * wn;
    if (av) {
      // A w_k by the same recurrence, and the residual r_k = r_{k-1} - phi_k A w_k
      const double aa = first ? 0.0 : awolder[e];
      const double ab = first ? 0.0 : awold[e];
      const double awn = (av[e] - S.eps_old * aa - S.delta * ab) * ig;
      awnew[e] = awn;
      const double r = res[e] - S.phi * awn;
      res[e] = r;
      acc += r * r;
    }
  }
  if (av) {
    acc = bsum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
  }
}

// mark systems whose last step met the stopping test as done (after their x update)
__global__ void k_mr_retire(MState* __restrict__ st, int nsys, KGlobal* __restrict__ gl) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || gl->all_done) return;
  int rem = 0;
  for (int i = 0; i < nsys; ++i) {
    if (!st[i].done && st[i].pad) st[i].done = 1;
    rem += st[i].done ? 0 : 1;
  }
  gl->remaining = rem;
  gl->all_done = rem == 0;
}

// x and y (P^{-1} rhs) buffers: the driver rotates r / y / w buffers on the host
int solve_minres(svar_handle* h, const svar_solve_opts* o, int nrhs, const double* rhs, double* x,
                 svar_solve_info* info, hipStream_t st) {
  SVAR_TRY(ensure_krylov(h, nrhs, 1, st));
  auto& K = h->kry;
  const int nsys = K.plan.nsys;
  const int64_t n = K.ntot;
  std::vector<void*> tmp;
  double *R0 = nullptr, *R1 = nullptr, *R2 = nullptr, *W0 = nullptr, *W1 = nullptr, *W2 = nullptr,
         *v = nullptr;
  // two-norm test: A v, A w (three generations) and the carried residual
  const bool two = o->minres_norm == 0;
  double *AV = nullptr, *AW0 = nullptr, *AW1 = nullptr, *AW2 = nullptr, *RES = nullptr;
  MState* ms = nullptr;
  int rc = SVAR_OK;
  for (double** p : {&R0, &R1, &R2, &W0, &W1, &W2, &v})
    if (rc == SVAR_OK) rc = dalloc(tmp, p, (size_t)n);
  if (two)
    for (double** p : {&AV, &AW0, &AW1, &AW2, &RES})
      if (rc == SVAR_OK) rc = dalloc(tmp, p, (size_t)n);
  if (rc == SVAR_OK) rc = dalloc(tmp, &ms, (size_t)nsys);
  if (rc != SVAR_OK) {
    free_all(tmp);
    return rc;
  }
  Program *PA = nullptr, *PP = nullptr;
  rc = get_program(h, PROG_A, nrhs, PV_F64, &PA, st);
  if (rc == SVAR_OK) rc = get_program(h, PROG_P, nrhs, PV_F64, &PP, st);
  std::vector<double> rhs2;
  if (rc == SVAR_OK) rc = sys_norm2(h, rhs, rhs2, st);
  int iters_done = 0;
  double* hist = (o->history && o->history_len > 0) ? o->history : nullptr;
  const int hlen = hist ? o->history_len : 0;
  if (rc == SVAR_OK) {
    launch_fill(x, n, 0.0, st);
    if (hist)
      launch_fill(hist, (int64_t)nsys * hlen, std::numeric_limits<double>::quiet_NaN(), st);
    // the first steps read the older search directions scaled by zero: keep them finite
    for (double* p : {W0, W1, W2, AW0, AW1, AW2})
      if (p) launch_fill(p, n, 0.0, st);
    if (two)
      (void)hipMemcpyAsync(RES, rhs, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    // r = rhs, y = P^{-1} r, beta_1^2 = r^T y
    double* r_prev = R0;
    double* r = R1;
    double* y = R2;
    (void)hipMemcpyAsync(r, rhs, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    rc = run_program(h, *PP, r, y, st, nullptr);
    hipLaunchKernelGGL(k_mr_dot, dim3(K.plan.ntask), dim3(NT), 0, st, K.plan.tasks, r, y, K.npart);
    kr_seg_sum(K.plan, K.npart, K.sysv, st);
    // rhs norms for the two-norm test (the host copy rhs2 is uploaded into K.tol_rel)
    (void)hipMemcpyAsync(K.tol_rel, rhs2.data(), nsys * sizeof(double), hipMemcpyHostToDevice, st);
    hipLaunchKernelGGL(k_mr_init, dim3(1), dim3(64), 0, st, ms, K.sysv, K.tol_rel, o->rtol, nsys,
                       K.gl);
    double* wolder = W0;
    double* wold = W1;
    double* wnew = W2;
    const int* skip = &K.gl->all_done;
    for (int k = 1; rc == SVAR_OK && k <= o->maxit; ++k) {
      hipLaunchKernelGGL(k_mr_v, dim3(K.plan.ntask), dim3(NT), 0, st, K.plan.tasks, ms, K.gl, y, v);
      rc = run_program(h, *PA, v, y, st, skip);  // y = A v
      if (rc != SVAR_OK) break;
      hipLaunchKernelGGL(k_mr_y1, dim3(K.plan.ntask), dim3(NT), 0, st, K.plan.tasks, ms, K.gl, y,
                         r_prev, v, k == 1 ? 1 : 0, K.npart, AV);
      kr_seg_sum(K.plan, K.npart, K.sysv, st);
      hipLaunchKernelGGL(k_mr_y2, dim3(K.plan.ntask), dim3(NT), 0, st, K.plan.tasks, K.plan.sys, ms,
                         K.gl, K.sysv, y, r);
      // rotate: r_prev <- r, r <- y, y <- free buffer
      double* freebuf = r_prev;
      r_prev = r;
      r = y;
      y = freebuf;
      rc = run_program(h, *PP, r, y, st, skip);  // y = P^{-1} r
      if (rc != SVAR_OK) break;
      hipLaunchKernelGGL(k_mr_dot, dim3(K.plan.ntask), dim3(NT), 0, st, K.plan.tasks, r, y,
                         K.npart);
      kr_seg_sum(K.plan, K.npart, K.sysv, st);
      hipLaunchKernelGGL(k_mr_scalar, dim3((nsys + 63) / 64), dim3(64), 0, st, ms, K.sysv, nsys,
                         K.gl, two ? 0 : 1, hist, hlen);
      hipLaunchKernelGGL(k_mr_w, dim3(K.plan.ntask), dim3(NT), 0, st, K.plan.tasks, K.plan.sys, ms,
                         K.gl, v, wolder, wold, wnew, x, k == 1 ? 1 : 0, AV, AW0, AW1, AW2, RES,
                         K.npart);
      if (two) {
        kr_seg_sum(K.plan, K.npart, K.sysv, st);
        hipLaunchKernelGGL(k_mr_check, dim3((nsys + 63) / 64), dim3(64), 0, st, ms, K.sysv, nsys,
                           K.gl, hist, hlen);
      }
      hipLaunchKernelGGL(k_mr_retire, dim3(1), dim3(64), 0, st, ms, nsys, K.gl);
      double* t0 = wolder;
      wolder = wold;
      wold = wnew;
      wnew = t0;
      double* a0 = AW0;
      AW0 = AW1;
      AW1 = AW2;
      AW2 = a0;
      iters_done = k;
      if (k % 8 == 0 || k == o->maxit) {
        if (hipMemcpyAsync(K.gl_host, K.gl, sizeof(KGlobal), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
          rc = SVAR_E_HIP;
          break;
        }
        if (K.gl_host->all_done) break;
      }
    }
  }
  (void)iters_done;
  std::vector<MState> hs(nsys);
  if (rc == SVAR_OK) {
    if (hipMemcpyAsync(hs.data(), ms, nsys * sizeof(MState), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = SVAR_E_HIP;
  }
  std::vector<double> r2;
  if (rc == SVAR_OK) {
    rc = run_program(h, *PA, x, K.r, st, nullptr);
    kr_resid(K.r, rhs, n, st);
    if (rc == SVAR_OK) rc = sys_norm2(h, K.r, r2, st);
  }
  if (rc == SVAR_OK) {
    const double sc = 1.0 / (double)nsys;
    for (int i = 0; i < nsys; ++i) {
      svar_solve_info& I = info[i];
      const double nb = std::sqrt(rhs2[i]);
      I.iters = hs[i].iters;
      I.outer = 1;
      I.relres_true = nb > 0 ? std::sqrt(r2[i]) / nb : 0.0;
      I.relres_est = two ? (nb > 0 ? hs[i].res2 / nb : 0.0)
                         : (hs[i].beta1 > 0 ? hs[i].phibar / hs[i].beta1 : 0.0);
      I.status = hs[i].status;
      if (I.status == SVAR_OK && !hs[i].done && hs[i].pad == 0) I.status = SVAR_E_NOCONV;
      // rtol is a two-norm tolerance whatever the stopping rule: a P^{-1}-norm stop with a
      // larger true residual, or a carried residual that drifted from the true one, is not OK
      if (I.status == SVAR_OK && !(I.relres_true <= o->rtol))
        I.status = std::isfinite(I.relres_true) ? SVAR_E_NOCONV : SVAR_E_BREAKDOWN;
      const int it = hs[i].iters;
      I.n_M = (int64_t)std::llround((PA->cnt[0] + PP->cnt[0]) * sc * it + PA->cnt[0] * sc);
      I.n_MT = (int64_t)std::llround((PA->cnt[1] + PP->cnt[1]) * sc * it + PA->cnt[1] * sc);
      I.n_D = (int64_t)std::llround((PA->cnt[2] + PP->cnt[2]) * sc * it + PA->cnt[2] * sc);
      I.n_R = (int64_t)std::llround((PA->cnt[3] + PP->cnt[3]) * sc * it + PA->cnt[3] * sc);
      I.n_Rhat_inv = (int64_t)std::llround(PP->cnt[4] * sc * (it + 1));
      I.n_Dhat_inv = (int64_t)std::llround(PP->cnt[5] * sc * (it + 1));
      if (I.status != SVAR_OK && rc == SVAR_OK) rc = I.status;
    }
    if (rc != SVAR_OK) set_error("at least one system did not converge (see info)");
  }
  (void)hipStreamSynchronize(st);
  free_all(tmp);
  return rc;
}

}  // namespace svar
