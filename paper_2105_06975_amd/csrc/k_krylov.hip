// Device-resident flexible GMRES (right preconditioned, x0 = 0 per cycle), float64.
//
// Many independent systems (windows x right-hand sides) advance in lock step; each has its
// own Hessenberg matrix, Givens rotations and convergence flag.  The iteration counter j is
// kept in device memory so that one iteration is the same sequence of launches every time.
//
// Orthogonalisation: classical Gram-Schmidt with the second (re-orthogonalisation) pass of
// each new vector delayed into the next iteration.  Iteration j holds u_j, the candidate for
// v_j after one projection, scaled to unit norm, and uses it directly as the input of the
// preconditioner (flexible GMRES accepts any z_j; A Z = V Hbar stays exact).  With
// w = A P^{-1} u_j, one pass over V_{0..j-1} computes V^T w, V^T u_j, u_j^T w, u_j^T u_j; then
//   v_j = (u_j - V s)/nu,  s = V^T u_j,  nu^2 = u_j^T u_j - s^T s,
//   column j-1 of Hbar = (h_{j-1} + s/sigma_j, nu/sigma_j)    (sigma_j: scale applied to u_j),
//   provisional column j: h_t = (V^T w)_t, h_j = (u_j^T w - s^T V^T w)/nu,
// and a second pass writes v_j and u_{j+1} = w - V h - v_j h_j.  Two reads of the basis per
// iteration instead of four for two-pass classical Gram-Schmidt.
#include "svar_impl.h"
#include "krylov.h"
#include "lanes.h"

namespace svar {

static constexpr int NT = 256;

// wave sums without the LDS crossbar (lanes.h); wave_sum16 leaves the wave total of value
// (l >> 2) & 15 in lane l
using lanes::wave_sum;
using lanes::wave_sum16;

// block-wide sum of one value per thread; every thread gets the result
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  __syncthreads();
  if (ln == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  return t;
}

// ---------------------------------------------------------------- norms
__global__ __launch_bounds__(NT) void k_nrm2_part(const KTask* __restrict__ tasks,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ part) {
  __shared__ double red[NT / 64];
  const KTask t = tasks[blockIdx.x];
  double acc = 0.0;
  for (int64_t e = t.e0 + threadIdx.x; e < t.e1; e += NT) acc += x[e] * x[e];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// per-system sum of task partials (fixed order)
__global__ __launch_bounds__(64) void k_seg_sum(const KSys* __restrict__ sys,
                                                const double* __restrict__ part,
                                                double* __restrict__ out) {
  const KSys S = sys[blockIdx.x];
  double acc = 0.0;
  for (int i = threadIdx.x; i < S.ntask; i += 64) acc += part[S.task0 + i];
  acc = wave_sum(acc);
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// ---------------------------------------------------------------- cycle start
// u = r / ||r|| per system; state reset; global j = 0.
__global__ __launch_bounds__(NT) void k_fg_start(const KTask* __restrict__ tasks,
                                                 const KSys* __restrict__ sys,
                                                 const double* __restrict__ part,
                                                 const double* __restrict__ r,
                                                 double* __restrict__ u, KState* __restrict__ st,
                                                 const double* __restrict__ tol_rel,
                                                 KGlobal* __restrict__ gl, int nsys) {
  __shared__ double red[NT / 64];
  const KTask t = tasks[blockIdx.x];
  const KSys S = sys[t.sys];
  double acc = 0.0;
  for (int i = threadIdx.x; i < S.ntask; i += NT) acc += part[S.task0 + i];
  const double nrm = sqrt(block_sum(acc, red));
  const bool zero = !(nrm > 0.0);
  const double sig = zero ? 0.0 : 1.0 / nrm;
  for (int64_t e = t.e0 + threadIdx.x; e < t.e1; e += NT) u[e] = r[e] * sig;
  if (threadIdx.x == 0 && blockIdx.x == (unsigned)S.task0) {
    KState s0;
    s0.done = (zero || tol_rel[t.sys] >= 1.0) ? 1 : 0;  // tol_rel >= 1: inactive system
    s0.iters = 0;
    s0.status = isfinite(nrm) ? 0 : SVAR_E_BREAKDOWN;
    if (!isfinite(nrm)) s0.done = 1;
    s0.fallback = 0;
    s0.stall = 0;
    s0.pad2 = 0;
    s0.beta = nrm;
    s0.tol_abs = tol_rel[t.sys] * nrm;
    s0.sigma = sig;
    s0.nu = 0.0;
    s0.est = nrm;
    st[t.sys] = s0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    gl->j = 0;
    gl->remaining = nsys;  // corrected by k_fg_count
  }
}

// count systems that are already done at the start of a cycle
__global__ void k_fg_count(const KState* __restrict__ st, KGlobal* __restrict__ gl, int nsys) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int rem = 0;
    for (int i = 0; i < nsys; ++i) rem += st[i].done ? 0 : 1;
    gl->remaining = rem;
    gl->all_done = rem == 0 ? 1 : 0;
  }
}

// u *= 1 / ||u|| (norm from the update pass partials); sigma recorded; j advanced.
__global__ __launch_bounds__(NT) void k_fg_scale(const KTask* __restrict__ tasks,
                                                 const KSys* __restrict__ sys,
                                                 const double* __restrict__ part,
                                                 double* __restrict__ u, KState* __restrict__ st,
                                                 KGlobal* __restrict__ gl) {
  __shared__ double red[NT / 64];
  if (gl->all_done) return;
  const KTask t = tasks[blockIdx.x];
  const KSys S = sys[t.sys];
  if (st[t.sys].done) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < S.ntask; i += NT) acc += part[S.task0 + i];
  const double nrm = sqrt(block_sum(acc, red));
  const double sig = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t e = t.e0 + threadIdx.x; e < t.e1; e += NT) u[e] *= sig;
  if (threadIdx.x == 0 && blockIdx.x == (unsigned)S.task0) st[t.sys].sigma = sig;
}

// The basis is streamed once per pass and not reused before the next pass: its loads are
// non-temporal (measured: 3 % less Gram-Schmidt time at C2 x 8 rhs).

// ---------------------------------------------------------------- dot pass
// partial sums per task: [0, j) V^T w, [m, m+j) V^T u, 2m: u^T w, 2m+1: u^T u.
// Also stores z into Z[j].  Each thread keeps its EPT elements of u and w in registers.
template <int EPT>
__global__ __launch_bounds__(NT) void k_fg_dot(const KTask* __restrict__ tasks,
                                               const KState* __restrict__ st,
                                               const KGlobal* __restrict__ gl,
                                               const double* __restrict__ V,
                                               const double* __restrict__ u,
                                               const double* __restrict__ w,
                                               const double* __restrict__ z,
                                               double* __restrict__ Zb, int64_t ntot, int m,
                                               int with_w, double* __restrict__ part) {
  __shared__ double lw[NT / 64][64];
  __shared__ double lu[NT / 64][64];
  if (gl->all_done) return;
  const KTask t = tasks[blockIdx.x];
  if (st[t.sys].done) return;
  const int j = gl->j;
  const int SL = 2 * m + 2;
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  double ur[EPT], wr[EPT];
  int64_t idx[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    idx[q] = t.e0 + threadIdx.x + (int64_t)q * NT;
    const bool ok = idx[q] < t.e1;
    ur[q] = ok ? u[idx[q]] : 0.0;
    wr[q] = (ok && with_w) ? w[idx[q]] : 0.0;
    if (ok && with_w) Zb[(int64_t)j * ntot + idx[q]] = z[idx[q]];
  }
  double* P = part + (int64_t)blockIdx.x * SL;
  int64_t cidx[EPT];  // clamped indices: loads stay in range, the weights are zero outside
#pragma unroll
  for (int q = 0; q < EPT; ++q) cidx[q] = idx[q] < t.e1 ? idx[q] : t.e1 - 1;
  for (int t0 = 0; t0 < j; t0 += 64) {
    const int tn = min(64, j - t0);
    for (int tt = 0; tt < tn; tt += 8) {
      double acc[16];
#pragma unroll
      for (int v8 = 0; v8 < 8; ++v8) {
        const int tv = min(t0 + tt + v8, j - 1);
        const double* Vt = V + (int64_t)tv * ntot;
        double aw = 0.0, au = 0.0;
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
          const double v = __builtin_nontemporal_load(Vt + cidx[q]);
          aw += v * wr[q];
          au += v * ur[q];
        }
        acc[2 * v8] = aw;
        acc[2 * v8 + 1] = au;
      }
      const double s = wave_sum16(acc);
      const int id = (ln >> 2) & 15;
      if ((ln & 3) == 0 && tt + (id >> 1) < tn) {
        if (id & 1)
          lu[wv][tt + (id >> 1)] = s;
        else
          lw[wv][tt + (id >> 1)] = s;
      }
    }
    __syncthreads();
    if (threadIdx.x < tn) {
      double a = 0.0, c = 0.0;
      for (int i = 0; i < NT / 64; ++i) {
        a += lw[i][threadIdx.x];
        c += lu[i][threadIdx.x];
      }
      P[t0 + threadIdx.x] = a;
      P[m + t0 + threadIdx.x] = c;
    }
    __syncthreads();
  }
  double uw = 0.0, uu = 0.0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    uw += ur[q] * wr[q];
    uu += ur[q] * ur[q];
  }
  uw = wave_sum(uw);
  uu = wave_sum(uu);
  if (ln == 0) {
    lw[wv][0] = uw;
    lu[wv][0] = uu;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int i = 0; i < NT / 64; ++i) {
      a += lw[i][0];
      c += lu[i][0];
    }
    P[2 * m] = a;
    P[2 * m + 1] = c;
  }
}

// sums[sys][slot] = sum over the system's tasks of part[task][slot] (fixed order).
// grid: (nsys, ceil(nslot_used / 8)); block 256 = 8 slots x 32 task lanes.
__global__ __launch_bounds__(NT) void k_fg_reduce(const KSys* __restrict__ sys,
                                                  const KState* __restrict__ st,
                                                  const KGlobal* __restrict__ gl,
                                                  const double* __restrict__ part,
                                                  double* __restrict__ sums, int m) {
  __shared__ double red[8][33];
  if (gl->all_done) return;
  if (st[blockIdx.x].done) return;
  const KSys S = sys[blockIdx.x];
  const int j = gl->j;
  const int SL = 2 * m + 2;
  const int nused = 2 * j + 2;  // compact index -> slot
  const int sl = threadIdx.x >> 5, tl = threadIdx.x & 31;
  const int ci = blockIdx.y * 8 + sl;
  int slot = -1;
  if (ci < nused) slot = ci < j ? ci : (ci < 2 * j ? m + (ci - j) : 2 * m + (ci - 2 * j));
  double acc = 0.0;
  if (slot >= 0)
    for (int i = tl; i < S.ntask; i += 32) acc += part[(int64_t)(S.task0 + i) * SL + slot];
  red[sl][tl] = acc;
  __syncthreads();
  if (tl == 0 && slot >= 0) {
    double s = 0.0;
    for (int i = 0; i < 32; ++i) s += red[sl][i];
    sums[(int64_t)blockIdx.x * SL + slot] = s;
  }
}

// ---------------------------------------------------------------- small dense step
// One workgroup per system: finalise column j-1, Givens, convergence, coefficients for the
// update pass.  finalize_only: no new column (last iteration of a cycle).
__global__ __launch_bounds__(NT) void k_fg_small(KState* __restrict__ st, KGlobal* __restrict__ gl,
                                                 const double* __restrict__ sums,
                                                 KHess* __restrict__ hs, int m, int finalize_only,
                                                 int* __restrict__ net_off, double drop,
                                                 int patience, HistArg hist) {
  __shared__ double red[NT / 64];
  __shared__ double col[1];
  extern __shared__ double dyn[];  // 3 j + 1 doubles
  if (gl->all_done) return;
  KState S = st[blockIdx.x];
  const int j = gl->j;
  if (S.done) return;
  const int SL = 2 * m + 2;
  const double* sm = sums + (int64_t)blockIdx.x * SL;
  KHess Hh = hs[blockIdx.x];
  // s = V^T u, ss = s^T s, sa = s^T (V^T w)
  double ss = 0.0, sa = 0.0;
  for (int t = threadIdx.x; t < j; t += NT) {
    const double sv = sm[m + t];
    ss += sv * sv;
    sa += sv * sm[t];
    Hh.coef_s[t] = sv;
  }
  ss = block_sum(ss, red);
  sa = block_sum(sa, red);
  const double uu = sm[2 * m + 1], uw = sm[2 * m];
  const double nu2 = uu - ss;
  const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
  const double sig = S.sigma;
  // finalise column j-1: H[0..j-1][j-1] = hprev + s / sigma, H[j][j-1] = nu / sigma
  if (j >= 1) {
    double* Hc = Hh.H + (int64_t)(j - 1) * (m + 1);
    // stage the new column and the rotations in LDS; the rotation chain runs on one thread
    // with the running entry in a register
    double* lc = dyn;           // j + 1
    double* lcs = dyn + (j + 1);  // j
    double* lsn = lcs + j;        // j
    for (int t = threadIdx.x; t < j; t += NT) {
      lc[t] = Hh.hprev[t] + sm[m + t] / sig;
      lcs[t] = Hh.cs[t];
      lsn[t] = Hh.sn[t];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      lc[j] = nu / sig;
      double carry = lc[0];
      for (int i = 0; i < j - 1; ++i) {
        const double bq = lc[i + 1];
        lc[i] = lcs[i] * carry + lsn[i] * bq;
        carry = -lsn[i] * carry + lcs[i] * bq;
      }
      lc[j - 1] = carry;
      const double a = lc[j - 1], bq = lc[j];
      double rho = hypot(a, bq);
      double c = 1.0, s = 0.0;
      if (rho > 0.0) {
        c = a / rho;
        s = bq / rho;
      }
      Hh.cs[j - 1] = c;
      Hh.sn[j - 1] = s;
      lc[j - 1] = rho;
      lc[j] = 0.0;
      const double gj = Hh.g[j - 1];
      Hh.g[j] = -s * gj;
      Hh.g[j - 1] = c * gj;
      const double prev = S.est;
      S.est = fabs(Hh.g[j]);
      // learned preconditioner: `patience` steps in a row that do not reduce the least-
      // squares residual by the factor (1 - drop) switch the correction off for this system
      // from the next application on
      if (net_off && drop > 0.0 && !net_off[blockIdx.x]) {
        if (S.est < (1.0 - drop) * prev) {
          S.stall = 0;
        } else if (++S.stall >= patience) {
          net_off[blockIdx.x] = 1;
          S.fallback = 1;
        }
      }
      S.iters = j;
      if (hist.h) {
        const int t = hist.it0[blockIdx.x] + j - 1;
        if (t < hist.len) hist.h[(int64_t)blockIdx.x * hist.len + t] = S.est;
      }
      bool fin = isfinite(S.est) && isfinite(rho);
      if (!fin) {
        S.status = SVAR_E_BREAKDOWN;
        S.done = 1;
      } else if (S.est <= S.tol_abs || !(nu / sig > 1e-300) || rho == 0.0) {
        S.done = 1;  // converged, or happy breakdown (invariant Krylov space)
      } else if (finalize_only) {
        S.done = 1;  // cycle exhausted
        S.status = SVAR_E_NOCONV;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= j; t += NT) Hc[t] = lc[t];
  } else if (threadIdx.x == 0) {
    Hh.g[0] = nu / sig;  // r = (nu / sigma) v_0
    S.est = Hh.g[0];
  }
  __syncthreads();
  // provisional column j of w
  if (threadIdx.x == 0) {
    col[0] = nu > 0.0 ? (uw - sa) / nu : 0.0;
    if (!S.done && !(nu > 0.0)) {  // u_j vanished: Krylov space exhausted at j (j = 0 only)
      S.done = 1;
      S.iters = j;
    }
  }
  __syncthreads();
  if (!finalize_only) {
    for (int t = threadIdx.x; t < j; t += NT) Hh.hprev[t] = sm[t];
    if (threadIdx.x == 0) Hh.hprev[j] = col[0];
  }
  if (threadIdx.x == 0) {
    S.nu = nu;
    st[blockIdx.x] = S;
    if (S.done) {
      const int left = atomicSub(&gl->remaining, 1) - 1;
      if (left == 0) gl->all_done = 1;
    }
  }
}

// ---------------------------------------------------------------- update pass
// v_j = (u - V s)/nu -> V[j];  u <- w - V h - v_j h_j;  partial ||u||^2 per task.
template <int EPT>
__global__ __launch_bounds__(NT) void k_fg_update(const KTask* __restrict__ tasks,
                                                  const KState* __restrict__ st,
                                                  const KGlobal* __restrict__ gl,
                                                  double* __restrict__ V, double* __restrict__ u,
                                                  const double* __restrict__ w,
                                                  const KHess* __restrict__ hs, int64_t ntot,
                                                  double* __restrict__ part) {
  extern __shared__ double coef[];  // [2 j + 1]: s_0..s_{j-1}, h_0..h_j
  __shared__ double red[NT / 64];
  if (gl->all_done) return;
  const KTask t = tasks[blockIdx.x];
  const KState S = st[t.sys];
  if (S.done) return;
  const int j = gl->j;
  const KHess Hh = hs[t.sys];
  for (int i = threadIdx.x; i < j; i += NT) coef[i] = Hh.coef_s[i];
  for (int i = threadIdx.x; i <= j; i += NT) coef[j + i] = Hh.hprev[i];
  __syncthreads();
  double as[EPT], ah[EPT];
  int64_t idx[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    idx[q] = t.e0 + threadIdx.x + (int64_t)q * NT;
    as[q] = 0.0;
    ah[q] = 0.0;
  }
  int64_t cidx[EPT];  // clamped: rows past the task end are computed but never stored
#pragma unroll
  for (int q = 0; q < EPT; ++q) cidx[q] = idx[q] < t.e1 ? idx[q] : t.e1 - 1;
  int tt = 0;
  for (; tt + 4 <= j; tt += 4) {
    double v[4][EPT];
#pragma unroll
    for (int u4 = 0; u4 < 4; ++u4)
#pragma unroll
      for (int q = 0; q < EPT; ++q)
        v[u4][q] = __builtin_nontemporal_load(V + (int64_t)(tt + u4) * ntot + cidx[q]);
#pragma unroll
    for (int u4 = 0; u4 < 4; ++u4) {
      const double cs_ = coef[tt + u4], ch = coef[j + tt + u4];
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        as[q] += v[u4][q] * cs_;
        ah[q] += v[u4][q] * ch;
      }
    }
  }
  for (; tt < j; ++tt) {
    const double cs_ = coef[tt], ch = coef[j + tt];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const double v = __builtin_nontemporal_load(V + (int64_t)tt * ntot + cidx[q]);
      as[q] += v * cs_;
      ah[q] += v * ch;
    }
  }
  const double inu = 1.0 / S.nu, hj = coef[2 * j];
  double acc = 0.0;
  double* Vj = V + (int64_t)j * ntot;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    if (idx[q] < t.e1) {
      const double vj = (u[idx[q]] - as[q]) * inu;
      Vj[idx[q]] = vj;
      const double un = w[idx[q]] - ah[q] - vj * hj;
      u[idx[q]] = un;
      acc += un * un;
    }
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// advance the iteration counter (advance != 0) and refresh the skip flags of the operator
// programs: flags[0] = every system done, flags[1 + sys] = system sys done, flags[1 + nsys + w]
// = every right-hand side of window w done (one thread per window; systems are packed window
// by window, nrhs per window)
// net_off (nullable): bit 0 = the learned correction was switched off (fallback), bit 1 = the
// system is done; the network kernels skip a system when either is set
__global__ void k_fg_advance(KGlobal* __restrict__ gl, const KState* __restrict__ st,
                             int* __restrict__ flags, int* __restrict__ net_off, int nsys,
                             int nrhs, int advance) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w == 0) {
    if (advance && !gl->all_done) gl->j = gl->j + 1;
    if (flags) flags[0] = gl->all_done;
  }
  if (!flags || w * nrhs >= nsys) return;
  int all = 1;
  for (int r = 0; r < nrhs; ++r) {
    const int sy = w * nrhs + r;
    const int d = st[sy].done ? 1 : 0;
    flags[1 + sy] = d;
    if (net_off) net_off[sy] = (net_off[sy] & 1) | (d << 1);
    all &= d;
  }
  flags[1 + nsys + w] = all;
}

// ---------------------------------------------------------------- end of cycle
// y = R^{-1} g (upper triangular from the rotated Hessenberg), one workgroup per system;
// column-oriented back substitution: y_i = g_i / R_ii, then g_t -= R_ti y_i for t < i.
__global__ __launch_bounds__(NT) void k_fg_solve_y(const KState* __restrict__ st,
                                                   KHess* __restrict__ hs, int m) {
  extern __shared__ double gv[];
  const KState S = st[blockIdx.x];
  KHess Hh = hs[blockIdx.x];
  const int nc = S.iters;
  for (int t = threadIdx.x; t < nc; t += NT) gv[t] = Hh.g[t];
  __syncthreads();
  for (int i = nc - 1; i >= 0; --i) {
    const double* Ri = Hh.H + (int64_t)i * (m + 1);
    const double d = Ri[i];
    const double yi = d != 0.0 ? gv[i] / d : 0.0;
    __syncthreads();
    for (int t = threadIdx.x; t < i; t += NT) gv[t] -= Ri[t] * yi;
    if (threadIdx.x == 0) Hh.y[i] = yi;
    __syncthreads();
  }
}

// x += Z y over each system's used columns
__global__ __launch_bounds__(NT) void k_fg_xupdate(const KTask* __restrict__ tasks,
                                                   const KState* __restrict__ st,
                                                   const KHess* __restrict__ hs,
                                                   const double* __restrict__ Zb, int64_t ntot,
                                                   double* __restrict__ x) {
  extern __shared__ double yv[];
  const KTask t = tasks[blockIdx.x];
  const int nc = st[t.sys].iters;
  const KHess Hh = hs[t.sys];
  for (int i = threadIdx.x; i < nc; i += NT) yv[i] = Hh.y[i];
  __syncthreads();
  for (int64_t e = t.e0 + threadIdx.x; e < t.e1; e += NT) {
    double acc = 0.0;
    for (int c = 0; c < nc; ++c) acc += yv[c] * Zb[(int64_t)c * ntot + e];
    x[e] += acc;
  }
}

// r = rhs - r  (r holds A x on entry)
__global__ void k_resid(double* __restrict__ r, const double* __restrict__ rhs, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    r[i] = rhs[i] - r[i];
}

// ---------------------------------------------------------------- launchers
static unsigned capg(int64_t n) {
  int64_t g = (n + NT - 1) / NT;
  return (unsigned)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

void kr_nrm2_part(const KPlan& p, const double* x, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_nrm2_part, dim3(p.ntask), dim3(NT), 0, st, p.tasks, x, part);
}
void kr_seg_sum(const KPlan& p, const double* part, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_sum, dim3(p.nsys), dim3(64), 0, st, p.sys, part, out);
}
void kr_start(const KPlan& p, const double* part, const double* r, double* u, KState* stt,
              const double* tol_rel, KGlobal* gl, hipStream_t st) {
  hipLaunchKernelGGL(k_fg_start, dim3(p.ntask), dim3(NT), 0, st, p.tasks, p.sys, part, r, u, stt,
                     tol_rel, gl, p.nsys);
  hipLaunchKernelGGL(k_fg_count, dim3(1), dim3(64), 0, st, stt, gl, p.nsys);
}
void kr_scale(const KPlan& p, const double* part, double* u, KState* stt, KGlobal* gl,
              hipStream_t st) {
  hipLaunchKernelGGL(k_fg_scale, dim3(p.ntask), dim3(NT), 0, st, p.tasks, p.sys, part, u, stt, gl);
}
void kr_dot(const KPlan& p, const KState* stt, const KGlobal* gl, const double* V,
            const double* u, const double* w, const double* z, double* Zb, int64_t ntot, int m,
            int with_w, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_fg_dot<KR_EPT>, dim3(p.ntask), dim3(NT), 0, st, p.tasks, stt, gl, V, u, w,
                     z, Zb, ntot, m, with_w, part);
}
void kr_reduce(const KPlan& p, const KState* stt, const KGlobal* gl, const double* part,
               double* sums, int m, int jmax, hipStream_t st) {
  const int gy = (2 * jmax + 2 + 7) / 8;
  hipLaunchKernelGGL(k_fg_reduce, dim3(p.nsys, gy), dim3(NT), 0, st, p.sys, stt, gl, part, sums,
                     m);
}
void kr_small(const KPlan& p, KState* stt, KGlobal* gl, const double* sums, KHess* hs, int m,
              int finalize_only, int jmax, int* net_off, double drop, int patience,
              HistArg hist, hipStream_t st) {
  hipLaunchKernelGGL(k_fg_small, dim3(p.nsys), dim3(NT), (size_t)(3 * jmax + 4) * sizeof(double),
                     st, stt, gl, sums, hs, m, finalize_only, net_off, drop,
                     patience < 1 ? 1 : patience, hist);
}
void kr_update(const KPlan& p, const KState* stt, const KGlobal* gl, double* V, double* u,
               const double* w, const KHess* hs, int64_t ntot, double* part, int jmax,
               hipStream_t st) {
  hipLaunchKernelGGL(k_fg_update<KR_EPT>, dim3(p.ntask), dim3(NT),
                     (size_t)(2 * jmax + 2) * sizeof(double), st, p.tasks, stt, gl, V, u, w, hs,
                     ntot, part);
}
void kr_advance(KGlobal* gl, const KState* stt, int* flags, int* net_off, int nsys, int nrhs,
                int advance, hipStream_t st) {
  const int nwin = flags ? (nsys + nrhs - 1) / nrhs : 1;
  hipLaunchKernelGGL(k_fg_advance, dim3((nwin + 255) / 256), dim3(256), 0, st, gl, stt, flags,
                     net_off, nsys, nrhs, advance);
}
void kr_solve_y(const KPlan& p, const KState* stt, KHess* hs, int m, hipStream_t st) {
  hipLaunchKernelGGL(k_fg_solve_y, dim3(p.nsys), dim3(NT), (size_t)(m + 1) * sizeof(double), st,
                     stt, hs, m);
}
void kr_xupdate(const KPlan& p, const KState* stt, const KHess* hs, const double* Zb,
                int64_t ntot, double* x, int m, hipStream_t st) {
  hipLaunchKernelGGL(k_fg_xupdate, dim3(p.ntask), dim3(NT), (size_t)(m + 1) * sizeof(double), st,
                     p.tasks, stt, hs, Zb, ntot, x);
}
// ================================================================ s-step (block) FGMRES
// A block of b columns starts from the last orthonormal basis vector v_j: z_{j+i} =
// P^{-1} w_i with w_0 = v_j and w_{i+1} = A z_{j+i} / d_i, d_i = ||A z_{j+i}||.  The block
// W = [w_1..w_b] (basis slots j+1..j+b) is projected out of V_{0..j} twice (block classical
// Gram-Schmidt with re-orthogonalisation, C = C1 + C2) and orthonormalised by two Cholesky QR
// rounds (W = Q R, R = R2 R1).  Then A z_{j+i} = d_i (V C e_i + Q R e_i): column j+i of Hbar
// holds d_i C[:, i] in rows 0..j and d_i R[0..i, i] in rows j+1..j+1+i, which is upper
// Hessenberg.  Four reads of V per block of b columns instead of two per column.  With a
// linear preconditioner the columns span the same Krylov space as one vector at a time.

// x *= 1 / ||x|| per system (norm from k_nrm2_part); the norm is kept as d_i of the block
__global__ __launch_bounds__(NT) void k_bk_scale(const KTask* __restrict__ tasks,
                                                 const KSys* __restrict__ sys,
                                                 const double* __restrict__ part,
                                                 double* __restrict__ x,
                                                 const KState* __restrict__ st,
                                                 const KGlobal* __restrict__ gl,
                                                 KBlock* __restrict__ kb, int i) {
  __shared__ double red[NT / 64];
  if (gl->all_done) return;
  const KTask t = tasks[blockIdx.x];
  if (st[t.sys].done) return;
  const KSys S = sys[t.sys];
  double acc = 0.0;
  for (int k = threadIdx.x; k < S.ntask; k += NT) acc += part[S.task0 + k];
  const double nrm = sqrt(block_sum(acc, red));
  const double sig = (nrm > 0.0 && isfinite(nrm)) ? 1.0 / nrm : 0.0;
  for (int64_t e = t.e0 + threadIdx.x; e < t.e1; e += NT) x[e] *= sig;
  if (threadIdx.x == 0 && blockIdx.x == (unsigned)S.task0) kb[t.sys].d[i] = nrm;
}

// partial sums per task of V_{0..j}^T W: part[task][t * B + i] (columns i >= b are zero)
template <int B>
__global__ __launch_bounds__(NT) void k_bk_dot(const KTask* __restrict__ tasks,
                                               const KState* __restrict__ st,
                                               const KGlobal* __restrict__ gl,
                                               const double* __restrict__ V, int64_t ldv, int j,
                                               int b, int SLB, double* __restrict__ part) {
  constexpr int EPT = KR_EPT;
  constexpr int TB = 16 / B;  // basis vectors per exchange batch (16 sums)
  constexpr int TW = 64 / B;  // basis vectors per LDS window
  __shared__ double lr[NT / 64][64];
  if (gl->all_done) return;
  const KTask t = tasks[blockIdx.x];
  if (st[t.sys].done) return;
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const int len = (int)(t.e1 - t.e0);
  const double* V0 = V + t.e0;
  const double* W0 = V0 + (int64_t)(j + 1) * ldv;
  int cidx[EPT];
  double wr[B][EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int o = (int)threadIdx.x + q * NT;
    cidx[q] = min(o, len - 1);
#pragma unroll
    for (int i = 0; i < B; ++i)
      wr[i][q] = (o < len && i < b) ? W0[(int64_t)i * ldv + cidx[q]] : 0.0;
  }
  double* P = part + (int64_t)blockIdx.x * SLB;
  const int nv = j + 1;
  for (int t0 = 0; t0 < nv; t0 += TW) {
    const int tn = min(TW, nv - t0);
    for (int tt = 0; tt < tn; tt += TB) {
      double acc[16];
#pragma unroll
      for (int v = 0; v < TB; ++v) {
        const double* Vt = V0 + (int64_t)min(t0 + tt + v, nv - 1) * ldv;
        double a[B];
#pragma unroll
        for (int i = 0; i < B; ++i) a[i] = 0.0;
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
          const double x = __builtin_nontemporal_load(Vt + cidx[q]);
#pragma unroll
          for (int i = 0; i < B; ++i) a[i] += x * wr[i][q];
        }
#pragma unroll
        for (int i = 0; i < B; ++i) acc[v * B + i] = a[i];
      }
      const double s = wave_sum16(acc);
      const int id = (ln >> 2) & 15, vv = id / B, ii = id - vv * B;
      if ((ln & 3) == 0 && tt + vv < tn) lr[wv][(tt + vv) * B + ii] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < tn * B) {
      double a = 0.0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) a += lr[w][threadIdx.x];
      P[t0 * B + threadIdx.x] = a;
    }
    __syncthreads();
  }
}

// sums[sys][slot] = sum over the system's tasks of part[task][slot], slot < nused (fixed
// order); grid (nsys, ceil(nused / 8)), 8 slots x 32 task lanes per workgroup
__global__ __launch_bounds__(NT) void k_bk_reduce(const KSys* __restrict__ sys,
                                                  const KState* __restrict__ st,
                                                  const KGlobal* __restrict__ gl,
                                                  const double* __restrict__ part, int SL,
                                                  int nused, double* __restrict__ sums) {
  __shared__ double red[8][33];
  if (gl->all_done) return;
  if (st[blockIdx.x].done) return;
  const KSys S = sys[blockIdx.x];
  const int sl = threadIdx.x >> 5, tl = threadIdx.x & 31;
  const int slot = blockIdx.y * 8 + sl;
  double acc = 0.0;
  if (slot < nused)
    for (int i = tl; i < S.ntask; i += 32) acc += part[(int64_t)(S.task0 + i) * SL + slot];
  red[sl][tl] = acc;
  __syncthreads();
  if (tl == 0 && slot < nused) {
    double s = 0.0;
    for (int i = 0; i < 32; ++i) s += red[sl][i];
    sums[(int64_t)blockIdx.x * SL + slot] = s;
  }
}

// W -= V_{0..j} C (C = the system's reduced sums, [t * B + i])
template <int B>
__global__ __launch_bounds__(NT) void k_bk_update(const KTask* __restrict__ tasks,
                                                  const KState* __restrict__ st,
                                                  const KGlobal* __restrict__ gl,
                                                  double* __restrict__ V, int64_t ldv, int j,
                                                  int b, int SLB, const double* __restrict__ C) {
  constexpr int EPT = KR_EPT;
  extern __shared__ double cf[];  // (j + 1) B
  if (gl->all_done) return;
  const KTask t = tasks[blockIdx.x];
  if (st[t.sys].done) return;
  const int nv = j + 1;
  const double* Cs = C + (int64_t)t.sys * SLB;
  for (int i = threadIdx.x; i < nv * B; i += NT) cf[i] = Cs[i];
  __syncthreads();
  const int len = (int)(t.e1 - t.e0);
  const double* V0 = V + t.e0;
  int cidx[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) cidx[q] = min((int)threadIdx.x + q * NT, len - 1);
  double acc[B][EPT];
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int q = 0; q < EPT; ++q) acc[i][q] = 0.0;
  int tt = 0;
  for (; tt + 2 <= nv; tt += 2) {
    double v[2][EPT];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < EPT; ++q)
        v[u][q] = __builtin_nontemporal_load(V0 + (int64_t)(tt + u) * ldv + cidx[q]);
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const double c = cf[(tt + u) * B + i];
#pragma unroll
        for (int q = 0; q < EPT; ++q) acc[i][q] += v[u][q] * c;
      }
  }
  for (; tt < nv; ++tt) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const double x = __builtin_nontemporal_load(V0 + (int64_t)tt * ldv + cidx[q]);
#pragma unroll
      for (int i = 0; i < B; ++i) acc[i][q] += x * cf[tt * B + i];
    }
  }
  double* W0 = V + t.e0 + (int64_t)(j + 1) * ldv;
#pragma unroll
  for (int i = 0; i < B; ++i) {
    if (i >= b) break;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int o = (int)threadIdx.x + q * NT;
      if (o < len) W0[(int64_t)i * ldv + o] -= acc[i][q];
    }
  }
}

// partial Gram matrix W^T W per task: part[task][i * B + l]
template <int B>
__global__ __launch_bounds__(NT) void k_bk_gram(const KTask* __restrict__ tasks,
                                                const KState* __restrict__ st,
                                                const KGlobal* __restrict__ gl,
                                                const double* __restrict__ V, int64_t ldv, int j,
                                                int b, double* __restrict__ part) {
  constexpr int EPT = KR_EPT;
  constexpr int NG = B * B;
  __shared__ double lr[NT / 64][64];
  if (gl->all_done) return;
  const KTask t = tasks[blockIdx.x];
  if (st[t.sys].done) return;
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const int len = (int)(t.e1 - t.e0);
  const double* W0 = V + t.e0 + (int64_t)(j + 1) * ldv;
  double wr[B][EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int o = (int)threadIdx.x + q * NT;
    const int c = min(o, len - 1);
#pragma unroll
    for (int i = 0; i < B; ++i) wr[i][q] = (o < len && i < b) ? W0[(int64_t)i * ldv + c] : 0.0;
  }
#pragma unroll
  for (int r0 = 0; r0 < NG; r0 += 16) {
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int g = r0 + u, i = g / B, l = g - i * B;
      double a = 0.0;
      if (g < NG) {
#pragma unroll
        for (int q = 0; q < EPT; ++q) a += wr[i][q] * wr[l][q];
      }
      acc[u] = a;
    }
    const double s = wave_sum16(acc);
    const int id = (ln >> 2) & 15;
    if ((ln & 3) == 0 && r0 + id < NG) lr[wv][r0 + id] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < NG) {
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) a += lr[w][threadIdx.x];
    part[(int64_t)blockIdx.x * NG + threadIdx.x] = a;
  }
}

// Cholesky factor of the block's Gram matrix (one thread per system): G = Rc^T Rc for the
// leading columns whose pivot keeps more than 1e-12 of the column's squared norm; round 0
// sets R = Rc and blen, round 1 sets R = Rc R and blen = min(blen, passing columns)
template <int B>
__global__ void k_bk_chol(const KState* __restrict__ st, const KGlobal* __restrict__ gl,
                          const double* __restrict__ gsum, KBlock* __restrict__ kb, int nsys,
                          int b, int round) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys || gl->all_done || st[s].done) return;
  const double* G = gsum + (int64_t)s * B * B;
  KBlock& K = kb[s];
  double R[B][B];
#pragma unroll
  for (int l = 0; l < B; ++l)
#pragma unroll
    for (int i = 0; i < B; ++i) R[l][i] = 0.0;
  int nb = 0;
  bool ok = true;
#pragma unroll
  for (int i = 0; i < B; ++i) {
    if (i < b && ok) {
#pragma unroll
      for (int l = 0; l < B; ++l) {
        if (l < i) {
          double v = G[l * B + i];
#pragma unroll
          for (int p = 0; p < B; ++p)
            if (p < l) v -= R[p][l] * R[p][i];
          R[l][i] = v / R[l][l];
        }
      }
      double piv = G[i * B + i];
#pragma unroll
      for (int p = 0; p < B; ++p)
        if (p < i) piv -= R[p][i] * R[p][i];
      if (piv > 1e-12 * G[i * B + i] && piv > 0.0 && isfinite(piv)) {
        R[i][i] = sqrt(piv);
        nb = i + 1;
      } else {
        ok = false;
      }
    }
  }
  // columns past the last passing one are not used: keep their factor entries finite
#pragma unroll
  for (int l = 0; l < B; ++l)
#pragma unroll
    for (int i = 0; i < B; ++i) {
      if (i >= nb) R[l][i] = (l == i) ? 1.0 : 0.0;
      K.Rc[l * B + i] = R[l][i];
    }
  if (round == 0) {
    K.blen = nb;
#pragma unroll
    for (int l = 0; l < B; ++l)
#pragma unroll
      for (int i = 0; i < B; ++i) K.R[l * B + i] = R[l][i];
  } else {
    K.blen = min(K.blen, nb);
    double P[B][B];
#pragma unroll
    for (int l = 0; l < B; ++l)
#pragma unroll
      for (int i = 0; i < B; ++i) {
        double v = 0.0;
#pragma unroll
        for (int p = 0; p < B; ++p) v += R[l][p] * K.R[p * B + i];
        P[l][i] = v;
      }
#pragma unroll
    for (int l = 0; l < B; ++l)
#pragma unroll
      for (int i = 0; i < B; ++i) K.R[l * B + i] = P[l][i];
  }
}

// W <- W Rc^{-1} over the leading blen columns (forward substitution per row)
template <int B>
__global__ __launch_bounds__(NT) void k_bk_trsm(const KTask* __restrict__ tasks,
                                                const KState* __restrict__ st,
                                                const KGlobal* __restrict__ gl,
                                                double* __restrict__ V, int64_t ldv, int j,
                                                int b, const KBlock* __restrict__ kb) {
  constexpr int EPT = KR_EPT;
  if (gl->all_done) return;
  const KTask t = tasks[blockIdx.x];
  if (st[t.sys].done) return;
  const KBlock& K = kb[t.sys];
  const int blen = min(K.blen, b);
  const int len = (int)(t.e1 - t.e0);
  double* W0 = V + t.e0 + (int64_t)(j + 1) * ldv;
  double w[B][EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int c = min((int)threadIdx.x + q * NT, len - 1);
#pragma unroll
    for (int i = 0; i < B; ++i) w[i][q] = i < blen ? W0[(int64_t)i * ldv + c] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < B; ++i) {
    if (i >= blen) break;
    const double inv = 1.0 / K.Rc[i * B + i];
#pragma unroll
    for (int l = 0; l < B; ++l) {
      if (l < i) {
        const double r = K.Rc[l * B + i];
#pragma unroll
        for (int q = 0; q < EPT; ++q) w[i][q] -= w[l][q] * r;
      }
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q) w[i][q] *= inv;
  }
#pragma unroll
  for (int i = 0; i < B; ++i) {
    if (i >= blen) break;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int o = (int)threadIdx.x + q * NT;
      if (o < len) W0[(int64_t)i * ldv + o] = w[i][q];
    }
  }
}

// The block's Hessenberg columns j..j+blen-1 of one system (one workgroup per system): built
// from C = S1 + S2, R and d in LDS; the rotations of earlier columns are applied to every new
// column at once (one thread per column), then the block's own rotations one column after
// the other; residual estimate, convergence and the learned-path stall test per column, as in
// the step-by-step kernel.  A block cut short by the Cholesky test, or the last block of the
// cycle, ends the system's cycle (the refinement loop restarts it from the true residual).
template <int B>
__global__ __launch_bounds__(NT) void k_bk_hess(KState* __restrict__ st, KGlobal* __restrict__ gl,
                                                const double* __restrict__ S1,
                                                const double* __restrict__ S2, int SLB,
                                                const KBlock* __restrict__ kbs,
                                                KHess* __restrict__ hs, int m, int j, int b,
                                                int* __restrict__ net_off, double drop,
                                                int patience, HistArg hist) {
  extern __shared__ double sm[];  // cs[j], sn[j], block cs/sn [2B], columns [b][j + b + 1]
  __shared__ int nused_s;
  if (gl->all_done) return;
  KState S = st[blockIdx.x];
  if (S.done) return;
  KHess Hh = hs[blockIdx.x];
  const KBlock& K = kbs[blockIdx.x];
  const int blen = min(K.blen, b);
  const int rows = j + b + 1;
  double* lcs = sm;
  double* lsn = sm + j;
  double* bcs = sm + 2 * j;
  double* bsn = bcs + B;
  double* col = bsn + B;
  const double* C1 = S1 + (int64_t)blockIdx.x * SLB;
  const double* C2 = S2 + (int64_t)blockIdx.x * SLB;
  for (int r = threadIdx.x; r < j; r += NT) {
    lcs[r] = Hh.cs[r];
    lsn[r] = Hh.sn[r];
  }
  for (int idx = threadIdx.x; idx < b * rows; idx += NT) {
    const int i = idx / rows, r = idx - i * rows;
    double v = 0.0;
    if (i < blen) {
      if (r <= j)
        v = (C1[r * B + i] + C2[r * B + i]) * K.d[i];
      else if (r - j - 1 <= i)
        v = K.R[(r - j - 1) * B + i] * K.d[i];
    }
    col[idx] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < blen && j > 0) {
    double* c = col + threadIdx.x * rows;
    double carry = c[0];
    for (int r = 0; r < j; ++r) {
      const double bq = c[r + 1];
      c[r] = lcs[r] * carry + lsn[r] * bq;
      carry = -lsn[r] * carry + lcs[r] * bq;
    }
    c[j] = carry;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (j == 0) Hh.g[0] = S.beta;  // r0 = beta v_0
    int used = 0;
    for (int i = 0; i < blen && !S.done; ++i) {
      const int c = j + i;
      double* cl = col + i * rows;
      double carry = cl[j];
      for (int r = j; r < c; ++r) {
        const double bq = cl[r + 1];
        cl[r] = bcs[r - j] * carry + bsn[r - j] * bq;
        carry = -bsn[r - j] * carry + bcs[r - j] * bq;
      }
      cl[c] = carry;
      const double a = cl[c], sub = cl[c + 1];
      const double rho = hypot(a, sub);
      double cs = 1.0, sn = 0.0;
      if (rho > 0.0) {
        cs = a / rho;
        sn = sub / rho;
      }
      bcs[i] = cs;
      bsn[i] = sn;
      cl[c] = rho;
      cl[c + 1] = 0.0;
      const double gj = Hh.g[c];
      Hh.g[c + 1] = -sn * gj;
      Hh.g[c] = cs * gj;
      const double prev = S.est;
      S.est = fabs(Hh.g[c + 1]);
      if (net_off && drop > 0.0 && !net_off[blockIdx.x]) {
        if (S.est < (1.0 - drop) * prev) {
          S.stall = 0;
        } else if (++S.stall >= patience) {
          net_off[blockIdx.x] = 1;
          S.fallback = 1;
        }
      }
      S.iters = c + 1;
      if (hist.h) {
        const int t = hist.it0[blockIdx.x] + c;
        if (t < hist.len) hist.h[(int64_t)blockIdx.x * hist.len + t] = S.est;
      }
      used = i + 1;
      if (!(isfinite(S.est) && isfinite(rho))) {
        S.status = SVAR_E_BREAKDOWN;
        S.done = 1;
      } else if (S.est <= S.tol_abs || !(fabs(sub) > 1e-300) || rho == 0.0) {
        S.done = 1;  // converged, or happy breakdown (invariant Krylov space)
      }
    }
    if (!S.done && (blen < b || j + b >= m)) {
      S.done = 1;  // cycle ended: block cut short or every basis slot used
      S.status = SVAR_E_NOCONV;
    }
    nused_s = used;
  }
  __syncthreads();
  const int used = nused_s;
  for (int idx = threadIdx.x; idx < used * rows; idx += NT) {
    const int i = idx / rows, r = idx - i * rows;
    if (r <= j + i + 1) Hh.H[(int64_t)(j + i) * (m + 1) + r] = col[idx];
  }
  for (int i = threadIdx.x; i < used; i += NT) {
    Hh.cs[j + i] = bcs[i];
    Hh.sn[j + i] = bsn[i];
  }
  if (threadIdx.x == 0) {
    st[blockIdx.x] = S;
    if (S.done) {
      const int left = atomicSub(&gl->remaining, 1) - 1;
      if (left == 0) gl->all_done = 1;
    }
  }
}

void kb_scale(const KPlan& p, const double* part, double* x, const KState* stt,
              const KGlobal* gl, KBlock* kb, int i, hipStream_t st) {
  hipLaunchKernelGGL(k_bk_scale, dim3(p.ntask), dim3(NT), 0, st, p.tasks, p.sys, part, x, stt, gl,
                     kb, i);
}
void kb_dot(int B, const KPlan& p, const KState* stt, const KGlobal* gl, const double* V,
            int64_t ldv, int j, int b, int SLB, double* part, hipStream_t st) {
  if (B == 4)
    hipLaunchKernelGGL(k_bk_dot<4>, dim3(p.ntask), dim3(NT), 0, st, p.tasks, stt, gl, V, ldv,
                       j, b, SLB, part);
  else
    hipLaunchKernelGGL(k_bk_dot<KB_MAX>, dim3(p.ntask), dim3(NT), 0, st, p.tasks, stt, gl, V,
                       ldv, j, b, SLB, part);
}
void kb_reduce(const KPlan& p, const KState* stt, const KGlobal* gl, const double* part, int SL,
               int nused, double* sums, hipStream_t st) {
  hipLaunchKernelGGL(k_bk_reduce, dim3(p.nsys, (nused + 7) / 8), dim3(NT), 0, st, p.sys, stt, gl,
                     part, SL, nused, sums);
}
void kb_update(int B, const KPlan& p, const KState* stt, const KGlobal* gl, double* V,
               int64_t ldv, int j, int b, int SLB, const double* C, hipStream_t st) {
  const size_t lds = (size_t)(j + 1) * B * sizeof(double);
  if (B == 4)
    hipLaunchKernelGGL(k_bk_update<4>, dim3(p.ntask), dim3(NT), lds, st, p.tasks, stt, gl, V,
                       ldv, j, b, SLB, C);
  else
    hipLaunchKernelGGL(k_bk_update<KB_MAX>, dim3(p.ntask), dim3(NT), lds, st, p.tasks, stt, gl,
                       V, ldv, j, b, SLB, C);
}
void kb_gram(int B, const KPlan& p, const KState* stt, const KGlobal* gl, const double* V,
             int64_t ldv, int j, int b, double* part, hipStream_t st) {
  if (B == 4)
    hipLaunchKernelGGL(k_bk_gram<4>, dim3(p.ntask), dim3(NT), 0, st, p.tasks, stt, gl, V, ldv, j,
                       b, part);
  else
    hipLaunchKernelGGL(k_bk_gram<KB_MAX>, dim3(p.ntask), dim3(NT), 0, st, p.tasks, stt, gl, V,
                       ldv, j, b, part);
}
void kb_chol(int B, const KPlan& p, const KState* stt, const KGlobal* gl, const double* gsum,
             KBlock* kb, int b, int round, hipStream_t st) {
  const dim3 g((p.nsys + 63) / 64), t(64);
  if (B == 4)
    hipLaunchKernelGGL(k_bk_chol<4>, g, t, 0, st, stt, gl, gsum, kb, p.nsys, b, round);
  else
    hipLaunchKernelGGL(k_bk_chol<KB_MAX>, g, t, 0, st, stt, gl, gsum, kb, p.nsys, b, round);
}
void kb_trsm(int B, const KPlan& p, const KState* stt, const KGlobal* gl, double* V, int64_t ldv,
             int j, int b, const KBlock* kb, hipStream_t st) {
  if (B == 4)
    hipLaunchKernelGGL(k_bk_trsm<4>, dim3(p.ntask), dim3(NT), 0, st, p.tasks, stt, gl, V, ldv, j,
                       b, kb);
  else
    hipLaunchKernelGGL(k_bk_trsm<KB_MAX>, dim3(p.ntask), dim3(NT), 0, st, p.tasks, stt, gl, V, ldv,
                       j, b, kb);
}
void kb_hess(int B, const KPlan& p, KState* stt, KGlobal* gl, const double* S1, const double* S2,
             int SLB, const KBlock* kb, KHess* hs, int m, int j, int b, int* net_off,
             double drop, int patience, HistArg hist, hipStream_t st) {
  const size_t lds = (size_t)(2 * j + 2 * B + b * (j + b + 1)) * sizeof(double);
  if (B == 4)
    hipLaunchKernelGGL(k_bk_hess<4>, dim3(p.nsys), dim3(NT), lds, st, stt, gl, S1, S2, SLB, kb, hs,
                       m, j, b, net_off, drop, patience < 1 ? 1 : patience, hist);
  else
    hipLaunchKernelGGL(k_bk_hess<KB_MAX>, dim3(p.nsys), dim3(NT), lds, st, stt, gl, S1, S2, SLB,
                       kb, hs, m, j, b, net_off, drop, patience < 1 ? 1 : patience, hist);
}

int kr_resident_tasks() {
  int dev = 0, cus = 0, a = 0, b = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_fg_dot<KR_EPT>, NT, 0) != hipSuccess)
    return 0;
  // the update pass's dynamic LDS (2 m + 2 doubles) is far below what limits its occupancy
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_fg_update<KR_EPT>, NT, 0) != hipSuccess)
    return 0;
  return cus * std::min(a, b);
}
void kr_resid(double* r, const double* rhs, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_resid, dim3(capg(n)), dim3(NT), 0, st, r, rhs, n);
}

}  // namespace svar
