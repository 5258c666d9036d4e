// Block flexible GMRES over the right-hand sides of a window (not in the paper: an algorithmic
// batching of its perturbed-observation right-hand sides, which share the saddle matrix).
//
// The P = nrhs residuals of window w form the block R_0 = V_0 S_0.  Block step j applies the
// preconditioner to every column of V_j (Z_j; flexible, so a nonlinear correction may enter),
// forms W = A Z_j, orthogonalises W against V_0..V_j by two passes (or one) of block classical
// Gram-Schmidt (C = C_1 + C_2) and factorises it by two Cholesky QR rounds on the
// column-normalised Gram matrix (W = V_{j+1} F, F = F_2 F_1 upper triangular).  The block
// Hessenberg matrix Hbar holds C in rows 0..(j+1)P-1 and F below, so that
// A [Z_0..Z_j] = [V_0..V_{j+1}] Hbar with P subdiagonals.  The least-squares problems
// min ||E_1 S_0 e_c - Hbar y_c|| share Hbar: Givens rotations (P per column, bottom up)
// triangularise it and rotate G = E_1 S_0, and column c's residual norm is the norm of rows
// (j+1)P..(j+2)P-1 of G e_c.  The cycle ends when every column of the window meets its
// tolerance or the basis is full; then X += [Z_0..Z_j] Y.
//
// Rank loss (a normalised Cholesky pivot <= 1e-14, or a zero column) is handled in two ways.
// In the starting block (a zero residual, two equal right-hand sides) the column's F row is
// zero, so R_0 = V_0 S_0 holds whatever that basis vector is: it is replaced by a seeded
// pseudo-random vector, which the second Cholesky QR round orthonormalises against the block
// (the basis then spans one more direction, which can only lower the least-squares residuals).
// In a later block it means the block Krylov space has become invariant up to rounding: the
// column is set to zero and the window's cycle ends after this step, so the least-squares
// problem never holds a zero column; the float64 restart continues from the true residual.
//
// Storage: a basis slot holds every system of the batch (windows one after another, the P
// right-hand sides of a window side by side, n rows each), so the block V_j of window w is P
// columns of slot j.  A task is a range of rows of one window; its threads keep their rows of
// all P columns in registers.
#include "krylov.h"
#include "lanes.h"
#include "svar_impl.h"

namespace svar {

static constexpr int NT = 256;
static constexpr int BR_EPT = KBR_TASK / NT;  // rows per thread of a task
static_assert(BR_EPT * NT == KBR_TASK, "a task is NT threads x BR_EPT rows");

using lanes::wave_sum16;

// packed address of column c, row e (inside the window) of task t's window
__device__ __forceinline__ int64_t bcol(const KBRTask& t, int c, int64_t e) {
  return t.off + (int64_t)c * t.n + e;
}

// seeded uniform value in [-1, 1) for row e of column c of window w (splitmix64 finaliser of
// the packed key)
__device__ __forceinline__ double bkr_rand(int w, int c, int64_t e) {
  uint64_t z = ((uint64_t)w << 40) ^ ((uint64_t)c << 36) ^ (uint64_t)e;
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

// the task's rows: thread rows e0 + threadIdx.x + q NT; rows past e1 are clamped (and masked)
struct BRows {
  int64_t e[BR_EPT];
  bool ok[BR_EPT];
  __device__ explicit BRows(const KBRTask& t) {
#pragma unroll
    for (int q = 0; q < BR_EPT; ++q) {
      const int64_t x = t.e0 + threadIdx.x + (int64_t)q * NT;
      ok[q] = x < t.e1;
      e[q] = ok[q] ? x : t.e1 - 1;
    }
  }
};

// Gram matrix partials of the task's rows: out[r P + c] = sum over the workgroup's rows of
// y[r] y[c] (rows outside the task hold zeros); wave sums, then the four waves in order
template <int P>
__device__ __forceinline__ void block_gram_part(const double (&y)[P][BR_EPT],
                                                double* __restrict__ out) {
  constexpr int PP = P * P;
  constexpr int NB = (PP + 15) / 16;
  __shared__ double lg[NT / 64][NB * 16];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
  for (int bt = 0; bt < NB; ++bt) {
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int v = bt * 16 + u;
      double x = 0.0;
      if (v < PP) {
        const int r = v / P, c = v % P;
#pragma unroll
        for (int q = 0; q < BR_EPT; ++q) x += y[r][q] * y[c][q];
      }
      acc[u] = x;
    }
    const double sm = wave_sum16(acc);
    if ((ln & 3) == 0) lg[wv][bt * 16 + (ln >> 2)] = sm;
  }
  __syncthreads();
  if ((int)threadIdx.x < PP) {
    double x = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) x += lg[k][threadIdx.x];
    out[threadIdx.x] = x;
  }
}

// Inner products of the P columns of na consecutive slots of A (slot s at A + s lda) with the
// P columns of the block at Wb: part[task][s P^2 + r P + c] = sum over the task's rows of
// A_s[col r] . W[col c].  V^T W of the Gram-Schmidt passes (A = V) and W^T W (A = Wb, na = 1).
template <int P>
__global__ __launch_bounds__(NT) void k_bkr_dot(const KBRTask* __restrict__ tasks,
                                                const KBRWin* __restrict__ wins,
                                                const double* __restrict__ A, int64_t lda, int na,
                                                const double* __restrict__ Wb,
                                                double* __restrict__ part, int SLP) {
  constexpr int PP = P * P;
  constexpr int NB = (PP + 15) / 16;  // exchange batches of 16 values
  __shared__ double lr[2][NT / 64][NB * 16];
  const KBRTask t = tasks[blockIdx.x];
  if (wins[t.win].done) return;
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const BRows R(t);
  double w[P][BR_EPT];
#pragma unroll
  for (int c = 0; c < P; ++c)
#pragma unroll
    for (int q = 0; q < BR_EPT; ++q) w[c][q] = R.ok[q] ? Wb[bcol(t, c, R.e[q])] : 0.0;
  double* out = part + (int64_t)blockIdx.x * SLP;
  for (int s = 0; s < na; ++s) {
    const double* As = A + (int64_t)s * lda;
    double a[P][BR_EPT];
#pragma unroll
    for (int r = 0; r < P; ++r)
#pragma unroll
      for (int q = 0; q < BR_EPT; ++q) a[r][q] = __builtin_nontemporal_load(As + bcol(t, r, R.e[q]));
    double(&L)[NT / 64][NB * 16] = lr[s & 1];
#pragma unroll
    for (int bt = 0; bt < NB; ++bt) {
      double acc[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int v = bt * 16 + u;
        double x = 0.0;
        if (v < PP) {
          const int r = v / P, c = v % P;
#pragma unroll
          for (int q = 0; q < BR_EPT; ++q) x += a[r][q] * w[c][q];
        }
        acc[u] = x;
      }
      const double sm = wave_sum16(acc);
      if ((ln & 3) == 0) L[wv][bt * 16 + (ln >> 2)] = sm;
    }
    __syncthreads();
    if ((int)threadIdx.x < PP) {
      double x = 0.0;
#pragma unroll
      for (int k = 0; k < NT / 64; ++k) x += L[k][threadIdx.x];
      out[s * PP + threadIdx.x] = x;
    }
  }
}

// sums[w][v] = sum over the window's tasks of part[task][v], v < nv (fixed order): a workgroup
// takes 32 values of one window, its 8 waves-of-32 sum every 8th task each (coalesced 256-byte
// reads of one task's 32 values), and the 8 partial sums are added in order through LDS
static constexpr int RV = 32, RG = NT / RV;
__global__ __launch_bounds__(NT) void k_bkr_reduce(const KBRWin* __restrict__ wins,
                                                   const double* __restrict__ part, int SLP,
                                                   int nv, double* __restrict__ sums, int SLS) {
  __shared__ double red[RG][RV];
  const int w = blockIdx.x;
  if (wins[w].done) return;
  const int task0 = wins[w].task0, ntask = wins[w].ntask;
  const int vl = threadIdx.x % RV, g = threadIdx.x / RV;
  const int v = blockIdx.y * RV + vl;
  double x = 0.0;
  if (v < nv)
    for (int k = g; k < ntask; k += RG) x += part[(int64_t)(task0 + k) * SLP + v];
  red[g][vl] = x;
  __syncthreads();
  if (g == 0 && v < nv) {
    double t = red[0][vl];
#pragma unroll
    for (int q = 1; q < RG; ++q) t += red[q][vl];
    sums[(int64_t)w * SLS + v] = t;
  }
}

// Wb[col c] += sgn sum_{s < na} sum_r A_s[col r] C[w][s P^2 + r P + c] over the task's rows.
// final_x: the solution update after the cycle (every window, na limited to its steps).  C is
// the same for the whole workgroup, so its entries come through scalar loads; a slot's P x 4
// basis values are loaded together before their FMAs.
template <int P>
__global__ __launch_bounds__(NT) void k_bkr_update(const KBRTask* __restrict__ tasks,
                                                   const KBRWin* __restrict__ wins,
                                                   const double* __restrict__ A, int64_t lda,
                                                   int na, double* __restrict__ Wb,
                                                   const double* __restrict__ C, int SLS,
                                                   double sgn, int final_x,
                                                   double* __restrict__ gpart, int SLP) {
  constexpr int PP = P * P;
  const KBRTask t = tasks[blockIdx.x];
  if (final_x) {
    na = min(na, wins[t.win].steps);
    if (na <= 0) return;
  } else if (wins[t.win].done) {
    return;
  }
  const double* __restrict__ Cw = C + (int64_t)t.win * SLS;
  const BRows R(t);
  // the block's own rows are loaded first, so that their latency overlaps the basis stream
  double acc[P][BR_EPT];
#pragma unroll
  for (int c = 0; c < P; ++c)
#pragma unroll
    for (int q = 0; q < BR_EPT; ++q) acc[c][q] = R.ok[q] ? Wb[bcol(t, c, R.e[q])] : 0.0;
  for (int s = 0; s < na; ++s) {
    const double* As = A + (int64_t)s * lda;
    const double* Cs = Cw + s * PP;
    double a[P][BR_EPT];
#pragma unroll
    for (int r = 0; r < P; ++r)
#pragma unroll
      for (int q = 0; q < BR_EPT; ++q) a[r][q] = __builtin_nontemporal_load(As + bcol(t, r, R.e[q]));
#pragma unroll
    for (int r = 0; r < P; ++r)
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const double cv = sgn * Cs[r * P + c];
#pragma unroll
        for (int q = 0; q < BR_EPT; ++q) acc[c][q] += a[r][q] * cv;
      }
  }
#pragma unroll
  for (int c = 0; c < P; ++c)
#pragma unroll
    for (int q = 0; q < BR_EPT; ++q) {
      if (R.ok[q]) Wb[bcol(t, c, R.e[q])] = acc[c][q];
      else acc[c][q] = 0.0;
    }
  // the Gram matrix of the updated block for the first Cholesky QR round
  if (gpart) block_gram_part<P>(acc, gpart + (int64_t)blockIdx.x * SLP);
}

// One Cholesky QR round of every active window's block from its Gram matrix G = W^T W:
// D = diag(sqrt(G_cc)), R^T R = D^{-1} G D^{-1} (Cholesky with deflation), F = R D; the
// rounds' product Ft <- F Ft (round 0: Ft = F).  A zero column, or a pivot <= 1e-14, deflates
// the column (R row zero, F_cc = 0): in round 0 of the starting block (start = 1) the trsm
// puts a random vector there, otherwise a zero one and the cycle ends after this step.  A
// non-finite G marks the window bad (breakdown).
template <int P>
__global__ void k_bkr_chol(KBRWin* __restrict__ wins, int nwin, const double* __restrict__ G,
                           int SLS, int round, int start) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwin) return;
  KBRWin& W = wins[w];
  if (W.done) return;
  const double* g = G + (int64_t)w * SLS;
  double d[P], R[P][P];
  int zm = 0;
  bool bad = false;
  for (int c = 0; c < P; ++c) {
    const double gc = g[c * P + c];
    if (!isfinite(gc)) bad = true;
    d[c] = gc > 0.0 ? sqrt(gc) : 0.0;
    if (!(d[c] > 0.0)) zm |= 1 << c;
    for (int i = 0; i < P; ++i) R[c][i] = 0.0;
  }
  for (int a = 0; a < P * P && !bad; ++a)
    if (!isfinite(g[a])) bad = true;
  if (bad) {
    W.bad = 1;
    return;
  }
  for (int j = 0; j < P; ++j) {
    if (zm >> j & 1) continue;
    double sj = 1.0;
    for (int k = 0; k < j; ++k) sj -= R[k][j] * R[k][j];
    if (!(sj > 1e-14)) {  // numerically dependent: deflate (R[k][j], k < j, stay)
      zm |= 1 << j;
      continue;
    }
    R[j][j] = sqrt(sj);
    for (int i = j + 1; i < P; ++i) {
      if (zm >> i & 1) continue;
      double v = g[j * P + i] / (d[j] * d[i]);
      for (int k = 0; k < j; ++k) v -= R[k][j] * R[k][i];
      R[j][i] = v / R[j][j];
    }
  }
  W.zmask = zm;
  W.rmask = (start && round == 0) ? zm : 0;
  if (zm && !start) W.cut = 1;
  double F[P][P];
  for (int i = 0; i < P; ++i)
    for (int j = 0; j < P; ++j) {
      F[i][j] = R[i][j] * d[j];
      W.Fr[i * P + j] = F[i][j];
    }
  if (round == 0) {
    for (int i = 0; i < P * P; ++i) W.Ft[i] = W.Fr[i];
  } else {
    double T[P * P];
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j) {
        double sm = 0.0;
        for (int k = i; k <= j; ++k) sm += F[i][k] * W.Ft[k * P + j];
        T[i * P + j] = sm;
      }
    for (int i = 0; i < P * P; ++i) W.Ft[i] = T[i];
  }
}

// W <- W F^{-1} row by row (F upper triangular); deflated columns become zero, or random
// (rmask).  gpart: also the Gram matrix partials of the result (the next Cholesky QR round).
template <int P>
__global__ __launch_bounds__(NT) void k_bkr_trsm(const KBRTask* __restrict__ tasks,
                                                 const KBRWin* __restrict__ wins,
                                                 double* __restrict__ Wb,
                                                 double* __restrict__ gpart, int SLP) {
  const KBRTask t = tasks[blockIdx.x];
  const KBRWin& W = wins[t.win];
  if (W.done || W.bad) return;
  __shared__ double f[P * P];
  if ((int)threadIdx.x < P * P) f[threadIdx.x] = W.Fr[threadIdx.x];
  const int zm = W.zmask, rm = W.rmask;
  __syncthreads();
  const BRows R(t);
  double y[P][BR_EPT];
#pragma unroll
  for (int q = 0; q < BR_EPT; ++q) {
#pragma unroll
    for (int c = 0; c < P; ++c) {
      double v = Wb[bcol(t, c, R.e[q])];
#pragma unroll
      for (int r = 0; r < c; ++r) v -= y[r][q] * f[r * P + c];
      y[c][q] = (zm >> c & 1) ? ((rm >> c & 1) ? bkr_rand(t.win, c, R.e[q]) : 0.0)
                              : v / f[c * P + c];
    }
  }
#pragma unroll
  for (int q = 0; q < BR_EPT; ++q)
#pragma unroll
    for (int c = 0; c < P; ++c) {
      if (R.ok[q]) Wb[bcol(t, c, R.e[q])] = y[c][q];
      else y[c][q] = 0.0;
    }
  if (gpart) block_gram_part<P>(y, gpart + (int64_t)blockIdx.x * SLP);
}

// every window's cycle state cleared before the QR of the starting block
__global__ void k_bkr_reset(KBRWin* __restrict__ wins, int nwin) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwin) return;
  wins[w].done = 0;
  wins[w].bad = 0;
  wins[w].steps = 0;
  wins[w].zmask = 0;
  wins[w].rmask = 0;
  wins[w].cut = 0;
}

// Cycle start (one thread per window): S_0 = Ft of the QR of R_0, G = E_1 S_0, per-column
// tolerances and states.  A window whose columns are all inactive (tol_rel >= 1) or whose R_0
// is not finite is done at once.
template <int P>
__global__ void k_bkr_start(KBRWin* __restrict__ wins, int nwin, const KBRHess* __restrict__ hs,
                            KState* __restrict__ st, const double* __restrict__ tol_rel,
                            const double* __restrict__ G0, int SLS, int m, KGlobal* gl) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < nwin) {
    KBRWin& W = wins[w];
    const KBRHess Hh = hs[w];
    const int ld = (m + 1) * P;
    bool active = false;
    for (int c = 0; c < P; ++c) active = active || tol_rel[w * P + c] < 1.0;
    W.done = (active && !W.bad) ? 0 : 1;
    W.stall = 0;
    double b2 = 0.0;
    for (int c = 0; c < P; ++c) b2 += fmax(G0[(int64_t)w * SLS + c * P + c], 0.0);
    W.prev = sqrt(b2);
    for (int c = 0; c < P; ++c)
      for (int r = 0; r < ld; ++r) Hh.G[(int64_t)c * ld + r] = (r < P) ? W.Ft[r * P + c] : 0.0;
    for (int c = 0; c < P; ++c) {
      const double beta = sqrt(fmax(G0[(int64_t)w * SLS + c * P + c], 0.0));
      KState S{};
      S.done = W.done;
      S.status = W.bad ? SVAR_E_BREAKDOWN : 0;
      S.beta = beta;
      S.tol_abs = tol_rel[w * P + c] * beta;
      S.est = beta;
      st[w * P + c] = S;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    gl->j = 0;
    gl->all_done = 0;
  }
}

// Block column j of Hbar for every active window (one workgroup per window): rows
// 0..(j+1)P-1 from the two Gram-Schmidt passes, F below; the earlier rotations; P new rotations
// per column; G rotated; per-column residuals, convergence and the window's state.
template <int P>
__global__ __launch_bounds__(64) void k_bkr_hess(KBRWin* __restrict__ wins,
                                                 const KBRHess* __restrict__ hs,
                                                 KState* __restrict__ st,
                                                 const double* __restrict__ C1,
                                                 const double* __restrict__ C2, int SLS, int j,
                                                 int m, int* __restrict__ net_off, double drop,
                                                 int patience, HistArg hist) {
  extern __shared__ double hc[];  // the block's P columns, ld rows each
  __shared__ double rc[P * P], rs[P * P], gl_[P][2 * P], est[P];
  __shared__ int okc[P];
  const int w = blockIdx.x;
  KBRWin& W = wins[w];
  if (W.done) return;
  const KBRHess Hh = hs[w];
  const int ld = (m + 1) * P;
  const int c = threadIdx.x;
  if (c < P) {
    double* col = hc + c * ld;
    for (int r = 0; r < ld; ++r) col[r] = 0.0;
    for (int s = 0; s <= j; ++s)
      for (int r = 0; r < P; ++r) {
        const int64_t v = (int64_t)w * SLS + s * P * P + r * P + c;
        col[s * P + r] = C2 ? C1[v] + C2[v] : C1[v];
      }
    for (int r = 0; r <= c; ++r) col[(j + 1) * P + r] = W.Ft[r * P + c];
    // rotations of the earlier block columns, in order (each acts on rows row, row + 1)
    for (int qq = 0; qq < j * P; ++qq)
      for (int k = 0; k < P; ++k) {
        const int row = qq + P - 1 - k;
        const double cs = Hh.cs[qq * P + k], sn = Hh.sn[qq * P + k];
        const double a = col[row], b = col[row + 1];
        col[row] = cs * a + sn * b;
        col[row + 1] = -sn * a + cs * b;
      }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int cc = 0; cc < P; ++cc) {
      const int qc = j * P + cc;
      double* cl = hc + cc * ld;
      for (int qq = 0; qq < cc; ++qq)  // rotations of the block's earlier columns
        for (int k = 0; k < P; ++k) {
          const int row = j * P + qq + P - 1 - k;
          const double cs = rc[qq * P + k], sn = rs[qq * P + k];
          const double a = cl[row], b = cl[row + 1];
          cl[row] = cs * a + sn * b;
          cl[row + 1] = -sn * a + cs * b;
        }
      for (int k = 0; k < P; ++k) {  // zero rows qc + P .. qc + 1, bottom up
        const int row = qc + P - 1 - k;
        const double a = cl[row], b = cl[row + 1];
        const double rho = hypot(a, b);
        double cs = 1.0, sn = 0.0;
        if (rho > 0.0) {
          cs = a / rho;
          sn = b / rho;
        }
        rc[cc * P + k] = cs;
        rs[cc * P + k] = sn;
        cl[row] = rho;
        cl[row + 1] = 0.0;
      }
    }
  }
  __syncthreads();
  // G: the block's rotations act on rows jP .. (j+2)P-1 only
  const int g = threadIdx.x;
  if (g < P) {
    double* Gc = Hh.G + (int64_t)g * ld;
    for (int r = 0; r < 2 * P; ++r) gl_[g][r] = Gc[j * P + r];
    for (int cc = 0; cc < P; ++cc)
      for (int k = 0; k < P; ++k) {
        const int row = cc + P - 1 - k;  // relative to jP
        const double cs = rc[cc * P + k], sn = rs[cc * P + k];
        const double x = gl_[g][row], y = gl_[g][row + 1];
        gl_[g][row] = cs * x + sn * y;
        gl_[g][row + 1] = -sn * x + cs * y;
      }
    double r2 = 0.0;
    for (int r = 0; r < 2 * P; ++r) {
      Gc[j * P + r] = gl_[g][r];
      if (r >= P) r2 += gl_[g][r] * gl_[g][r];
    }
    const double e = sqrt(r2);
    est[g] = e;
    KState S = st[w * P + g];
    S.est = e;
    S.iters = j + 1;
    okc[g] = isfinite(e) ? (e <= S.tol_abs ? 1 : 0) : -1;
    if (hist.h) {
      const int tt = hist.it0[w * P + g] + j;
      if (tt < hist.len) hist.h[(int64_t)(w * P + g) * hist.len + tt] = e;
    }
    st[w * P + g] = S;
  }
  // Hbar's new columns and the rotations back to global memory
  for (int v = threadIdx.x; v < P * ld; v += blockDim.x)
    Hh.H[(int64_t)(j * P) * ld + v] = hc[v];
  if ((int)threadIdx.x < P * P) {
    Hh.cs[(int64_t)(j * P) * P + threadIdx.x] = rc[threadIdx.x];
    Hh.sn[(int64_t)(j * P) * P + threadIdx.x] = rs[threadIdx.x];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bool all = true, fin = !W.bad;
    for (int q = 0; q < P; ++q) {
      if (okc[q] < 0) fin = false;
      if (okc[q] != 1) all = false;
    }
    W.steps = j + 1;
    // learned path: a step fails when the block's residual norm does not fall below
    // (1 - drop) times the previous one; after `patience` failures in a row the window's
    // systems apply the plain preconditioner from then on
    if (net_off && drop > 0.0) {
      double r2 = 0.0;
      for (int q = 0; q < P; ++q) r2 += est[q] * est[q];
      const double nrm = sqrt(r2);
      W.stall = (nrm < (1.0 - drop) * W.prev) ? 0 : W.stall + 1;
      W.prev = nrm;
      if (W.stall >= patience)
        for (int q = 0; q < P; ++q) {
          net_off[w * P + q] |= 1;
          st[w * P + q].fallback = 1;
        }
    }
    if (!fin || all || j + 1 >= m || W.cut) {
      W.done = 1;
      for (int q = 0; q < P; ++q) {
        KState S = st[w * P + q];
        S.done = 1;
        if (!fin) S.status = SVAR_E_BREAKDOWN;
        else if (!(est[q] <= S.tol_abs)) S.status = SVAR_E_NOCONV;
        st[w * P + q] = S;
      }
    }
  }
}

// Y = Rhat^{-1} G over the window's steps (back substitution; one thread per column), then
// Y in the update layout Yl[w][s P^2 + r P + c] = Y[c][s P + r]
template <int P>
__global__ __launch_bounds__(64) void k_bkr_solve_y(const KBRWin* __restrict__ wins,
                                                    const KBRHess* __restrict__ hs, int m,
                                                    double* __restrict__ Yl, int SLS) {
  const int w = blockIdx.x;
  const KBRWin& W = wins[w];
  const KBRHess Hh = hs[w];
  const int ld = (m + 1) * P;
  const int n = W.steps * P;
  const int g = threadIdx.x;
  if (g < P) {
    const double* G = Hh.G + (int64_t)g * ld;
    double* Y = Hh.Y + (int64_t)g * (m * P);
    for (int i = n - 1; i >= 0; --i) {
      double v = G[i];
      for (int k = i + 1; k < n; ++k) v -= Hh.H[(int64_t)k * ld + i] * Y[k];
      const double dg = Hh.H[(int64_t)i * ld + i];
      Y[i] = dg != 0.0 ? v / dg : 0.0;
    }
  }
  __syncthreads();
  for (int v = threadIdx.x; v < n * P; v += blockDim.x) {
    const int s = v / (P * P), r = (v / P) % P, cc = v % P;
    Yl[(int64_t)w * SLS + v] = Hh.Y[(int64_t)cc * (m * P) + s * P + r];
  }
}

// operator skip flags of the windows' systems, the network's done bits, the all-done flag
__global__ void k_bkr_flags(const KBRWin* __restrict__ wins, int nwin, int P,
                            KGlobal* __restrict__ gl, int* __restrict__ flags,
                            int* __restrict__ net_off) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < nwin) {
    const int d = wins[w].done ? 1 : 0;
    for (int r = 0; r < P; ++r) {
      flags[1 + w * P + r] = d;
      if (net_off) net_off[w * P + r] = (net_off[w * P + r] & 1) | (d << 1);
    }
    flags[1 + nwin * P + w] = d;
    if (!d) atomicAdd(&gl->remaining, 1);
  }
}
__global__ void k_bkr_count(KGlobal* __restrict__ gl, int* __restrict__ flags) {
  gl->all_done = gl->remaining == 0 ? 1 : 0;
  gl->j += 1;
  flags[0] = gl->all_done;
}
__global__ void k_bkr_clear(KGlobal* __restrict__ gl) { gl->remaining = 0; }

// ------------------------------------------------------------------ launchers
#define BKR_DISPATCH(P, CALL)                       \
  switch (P) {                                      \
    case 1: { constexpr int PT = 1; CALL; } break;  \
    case 2: { constexpr int PT = 2; CALL; } break;  \
    case 3: { constexpr int PT = 3; CALL; } break;  \
    case 4: { constexpr int PT = 4; CALL; } break;  \
    case 5: { constexpr int PT = 5; CALL; } break;  \
    case 6: { constexpr int PT = 6; CALL; } break;  \
    case 7: { constexpr int PT = 7; CALL; } break;  \
    default: { constexpr int PT = 8; CALL; } break; \
  }

void bkr_reset(const KBRPlan& p, KBRWin* wins, hipStream_t st) {
  hipLaunchKernelGGL(k_bkr_reset, dim3((p.nwin + 255) / 256), dim3(256), 0, st, wins, p.nwin);
}
void bkr_dot(int P, const KBRPlan& p, const KBRWin* wins, const double* A, int64_t lda, int na,
             const double* Wb, double* part, int SLP, hipStream_t st) {
  BKR_DISPATCH(P, hipLaunchKernelGGL(k_bkr_dot<PT>, dim3(p.ntask), dim3(NT), 0, st, p.tasks,
                                     wins, A, lda, na, Wb, part, SLP));
}
void bkr_reduce(const KBRPlan& p, const KBRWin* wins, const double* part, int SLP, int nv,
                double* sums, int SLS, hipStream_t st) {
  const int gy = (nv + RV - 1) / RV;
  hipLaunchKernelGGL(k_bkr_reduce, dim3(p.nwin, gy), dim3(NT), 0, st, wins, part, SLP, nv, sums,
                     SLS);
}
void bkr_update(int P, const KBRPlan& p, const KBRWin* wins, const double* A, int64_t lda,
                int na, double* Wb, const double* C, int SLS, double sgn, int final_x,
                double* gpart, int SLP, hipStream_t st) {
  BKR_DISPATCH(P, hipLaunchKernelGGL(k_bkr_update<PT>, dim3(p.ntask), dim3(NT), 0, st, p.tasks,
                                     wins, A, lda, na, Wb, C, SLS, sgn, final_x, gpart, SLP));
}
void bkr_chol(int P, const KBRPlan& p, KBRWin* wins, const double* G, int SLS, int round,
              int start, hipStream_t st) {
  BKR_DISPATCH(P, hipLaunchKernelGGL(k_bkr_chol<PT>, dim3((p.nwin + 63) / 64), dim3(64), 0, st,
                                     wins, p.nwin, G, SLS, round, start));
}
void bkr_trsm(int P, const KBRPlan& p, const KBRWin* wins, double* Wb, double* gpart, int SLP,
              hipStream_t st) {
  BKR_DISPATCH(P, hipLaunchKernelGGL(k_bkr_trsm<PT>, dim3(p.ntask), dim3(NT), 0, st, p.tasks,
                                     wins, Wb, gpart, SLP));
}
void bkr_start(int P, const KBRPlan& p, KBRWin* wins, KBRHess* hs, KState* stt,
               const double* tol_rel, const double* G0, int SLS, int m, KGlobal* gl,
               hipStream_t st) {
  BKR_DISPATCH(P, hipLaunchKernelGGL(k_bkr_start<PT>, dim3((p.nwin + 63) / 64), dim3(64), 0, st,
                                     wins, p.nwin, hs, stt, tol_rel, G0, SLS, m, gl));
}
void bkr_hess(int P, const KBRPlan& p, KBRWin* wins, KBRHess* hs, KState* stt, const double* C1,
              const double* C2, int SLS, int j, int m, int* net_off, double drop, int patience,
              HistArg hist, hipStream_t st) {
  const size_t sh = (size_t)P * (m + 1) * P * sizeof(double);
  BKR_DISPATCH(P, hipLaunchKernelGGL(k_bkr_hess<PT>, dim3(p.nwin), dim3(64), sh, st, wins, hs,
                                     stt, C1, C2, SLS, j, m, net_off, drop,
                                     patience < 1 ? 1 : patience, hist));
}
void bkr_solve_y(int P, const KBRPlan& p, const KBRWin* wins, const KBRHess* hs, int m,
                 double* Yl, int SLS, hipStream_t st) {
  BKR_DISPATCH(P, hipLaunchKernelGGL(k_bkr_solve_y<PT>, dim3(p.nwin), dim3(64), 0, st, wins, hs,
                                     m, Yl, SLS));
}
void bkr_flags(int P, const KBRPlan& p, const KBRWin* wins, KGlobal* gl, int* flags,
               int* net_off, hipStream_t st) {
  hipLaunchKernelGGL(k_bkr_clear, dim3(1), dim3(1), 0, st, gl);
  hipLaunchKernelGGL(k_bkr_flags, dim3((p.nwin + 255) / 256), dim3(256), 0, st, wins, p.nwin, P,
                     gl, flags, net_off);
  hipLaunchKernelGGL(k_bkr_count, dim3(1), dim3(1), 0, st, gl, flags);
}

}  // namespace svar
