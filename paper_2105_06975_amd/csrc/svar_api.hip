// libsvar host code: handle set-up, launch programs for A v and P^{-1} v, and the C ABI.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <numeric>

#include "setup.h"
#include "svar_handle.h"
#include "mem.h"

namespace svar {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

static int inval(const std::string& m) { return inval_msg(m); }

static int host_sum(const double* dpart, int n, hipStream_t st, double* out) {
  std::vector<double> hp(n);
  SVAR_HIP(hipMemcpyAsync(hp.data(), dpart, n * sizeof(double), hipMemcpyDeviceToHost, st));
  SVAR_HIP(hipStreamSynchronize(st));
  double s = 0.0;
  for (double v : hp) s += v;
  *out = s;
  return SVAR_OK;
}

// ------------------------------------------------------------------ GEMM planning
// Tasks: 64-row tiles x column groups x k-splits.  The k-range is split so that the launch
// has about four workgroups per CU; split partials are reduced in a fixed order.
static void plan_gemm(std::vector<GemmProb>& probs, std::vector<GemmTask>& tasks, int64_t& ws,
                      int& maxct, int target) {
  int maxcols = 1;
  for (auto& p : probs) maxcols = std::max(maxcols, p.ncols);
  maxct = std::min(8, (maxcols + 15) / 16);
  const int cw = maxct * 16;
  const int rows = 16 * gemm_rt(maxct);  // rows per workgroup
  double total_work = 0.0;
  for (auto& p : probs) total_work += (double)p.n * p.n * p.ncols;
  ws = 0;
  tasks.clear();
  for (int pi = 0; pi < (int)probs.size(); ++pi) {
    GemmProb& p = probs[pi];
    const int rtile = rows;
    const int rt = (p.n + rtile - 1) / rtile, cg = (p.ncols + cw - 1) / cw;
    const double share = total_work > 0 ? (double)p.n * p.n * p.ncols / total_work : 1.0;
    const int want = (int)std::ceil(target * share / (double)(rt * cg));
    const int kmin = 512;  // at least 128 k per wave
    const int maxs = std::max(1, p.n / kmin);
    int S = std::max(1, std::min(want, maxs));
    const int align = 64;
    const int chunk = ((p.n + S - 1) / S + align - 1) / align * align;
    S = (p.n + chunk - 1) / chunk;
    p.splits = S;
    p.ws_off = 0;
    if (S > 1) {
      p.ws_off = ws;
      ws += (int64_t)S * p.ncols * p.n;
    }
    for (int r = 0; r < rt; ++r)
      for (int sp = 0; sp < S; ++sp)
        for (int c = 0; c < cg; ++c) {
          GemmTask t;
          t.prob = pi;
          t.row0 = r * rtile;
          t.k0 = sp * chunk;
          t.k1 = std::min(p.n, (sp + 1) * chunk);
          t.col0 = c * cw;
          t.split = sp;
          tasks.push_back(t);
        }
  }
}

// Plan of the LDS-tiled kernel: 128-row x (16 maxct)-column tiles, split-K to fill `target`
// resident workgroups (CUs x workgroups per CU).
// Tasks that read the same panel chunk (same problem, k-range and column group) are placed on
// one XCD (workgroup i runs on XCD i mod 8), so the chunk is fetched into one L2 only.
static void plan_gemm_tiled(std::vector<GemmProb>& probs, std::vector<GemmTask>& tasks,
                            int64_t& ws, int& maxct, int target) {
  int maxcols = 1;
  for (auto& p : probs) maxcols = std::max(maxcols, p.ncols);
  // Column tile 16 ct and split-K chunk per problem.
  // One or two problems per launch (the single-window products): ct in 4..9 and one chunk
  // length chosen together so that the tasks fill whole rounds of the `target` resident
  // workgroups.  Estimated time = rounds x longest chunk (16-wide stages) x (ct + 2) (the MFMAs
  // and panel loads grow with ct, the matrix-row loads and the barrier do not) + one stage per
  // split (the partials' write and fixed-order reduce).  C2's D product (4096 x 520) on 512
  // slots: ct = 9, 32 x 4 tiles x 4 splits = 512 tasks in one round.
  // Many problems (a batch of uneven windows): the tile with the fewest padded columns
  // (ct 4..8, ties wider) and splits in proportion to each problem's share of the work, at
  // least 256 k per task.  A common short chunk there multiplies the tasks and the partial
  // tiles written for the reduce (64 C4 windows: 58 000 tasks against 3 300, +40 % GEMM time).
  const int rows = 128;
  const int np = (int)probs.size();
  std::vector<int> chunk(np), nsplit(np);
  if (np <= 2) {
    int maxst = 1;
    for (auto& p : probs) maxst = std::max(maxst, (p.n + 15) / 16);
    const int umin = std::min(maxst, 8);
    const int ctmax = std::min(9, std::max(2, (maxcols + 15) / 16));
    int bestU = maxst, bestct = ctmax;
    double bestcost = 1e300;
    for (int ct = std::min(4, ctmax); ct <= ctmax; ++ct) {
      const int cwt = 16 * ct;
      for (int U = maxst; U >= umin; --U) {
        int64_t ntask = 0;
        int longest = 0, maxS = 1;
        double wsb = 0.0;  // split-K partials (bytes)
        for (auto& p : probs) {
          const int st = (p.n + 15) / 16, S = (st + U - 1) / U, ch = (st + S - 1) / S;
          ntask += (int64_t)((p.n + rows - 1) / rows) * ((p.ncols + cwt - 1) / cwt) * S;
          longest = std::max(longest, ch);
          maxS = std::max(maxS, S);
          if (S > 1) wsb += 8.0 * S * p.ncols * (double)p.n;
        }
        // products with very wide panels (set-up inverses of large matrices) have tasks enough
        // without splits: keep their partials within 2 GiB (a 40,000^2 x 40,000 product would
        // otherwise ask for 20 splits' partials, 256 GB)
        if (wsb > 2147483648.0 && U < maxst) continue;
        const double cost =
            ((double)((ntask + target - 1) / target) * longest + maxS) * (ct + 2);
        if (cost < bestcost) {
          bestcost = cost;
          bestU = U;
          bestct = ct;
        }
      }
    }
    maxct = bestct;
    for (int pi = 0; pi < np; ++pi) {
      const int st = (probs[pi].n + 15) / 16, S = (st + bestU - 1) / bestU;
      chunk[pi] = 16 * ((st + S - 1) / S);
    }
  } else {
    int best = 8, bestpad = 1 << 30;
    for (int ct = 8; ct >= 4; --ct) {
      const int pad = (maxcols + 16 * ct - 1) / (16 * ct) * ct;
      if (pad < bestpad) {
        bestpad = pad;
        best = ct;
      }
    }
    maxct = std::min(best, (maxcols + 15) / 16);
    const int cwt = maxct * 16;
    double total_work = 0.0;
    for (auto& p : probs) total_work += (double)p.n * p.n * p.ncols;
    for (int pi = 0; pi < np; ++pi) {
      const GemmProb& p = probs[pi];
      const int rt = (p.n + rows - 1) / rows, cg = (p.ncols + cwt - 1) / cwt;
      const double share = total_work > 0 ? (double)p.n * p.n * p.ncols / total_work : 1.0;
      const int want = (int)std::ceil(target * share / (double)(rt * cg));
      const int S = std::max(1, std::min(want, std::max(1, p.n / 256)));
      chunk[pi] = ((p.n + S - 1) / S + 63) / 64 * 64;
    }
  }
  const int cw = maxct * 16;
  ws = 0;
  std::vector<std::vector<GemmTask>> groups;
  for (int pi = 0; pi < np; ++pi) {
    GemmProb& p = probs[pi];
    const int rt = (p.n + rows - 1) / rows, cg = (p.ncols + cw - 1) / cw;
    p.splits = (p.n + chunk[pi] - 1) / chunk[pi];
    p.ws_off = 0;
    if (p.splits > 1) {
      p.ws_off = ws;
      ws += (int64_t)p.splits * p.ncols * p.n;
    }
    for (int sp = 0; sp < p.splits; ++sp)
      for (int c = 0; c < cg; ++c) {
        std::vector<GemmTask> grp;
        for (int r = 0; r < rt; ++r) {
          GemmTask t;
          t.prob = pi;
          t.row0 = r * rows;
          t.k0 = sp * chunk[pi];
          t.k1 = std::min(p.n, (sp + 1) * chunk[pi]);
          t.col0 = c * cw;
          t.split = sp;
          grp.push_back(t);
        }
        groups.push_back(std::move(grp));
      }
  }
  // longest k-ranges first, so that the short tasks of small problems fill the last round of
  // resident workgroups instead of leaving long ones running alone at the end
  std::stable_sort(groups.begin(), groups.end(),
                   [](const std::vector<GemmTask>& a, const std::vector<GemmTask>& b) {
                     return (a[0].k1 - a[0].k0) > (b[0].k1 - b[0].k0);
                   });
  // deal the groups to 8 XCD queues (largest queue-balance first fit), then interleave
  const int NX = 8;
  std::vector<std::vector<GemmTask>> q(NX);
  for (auto& g : groups) {
    int best = 0;
    for (int x = 1; x < NX; ++x)
      if (q[x].size() < q[best].size()) best = x;
    q[best].insert(q[best].end(), g.begin(), g.end());
  }
  tasks.clear();
  std::vector<size_t> pos(NX, 0);
  size_t left = 0;
  for (auto& v : q) left += v.size();
  while (left > 0) {
    for (int x = 0; x < NX; ++x) {
      int src = x;
      if (pos[src] >= q[src].size()) {  // an exhausted queue: take from the fullest one
        src = 0;
        for (int y = 1; y < NX; ++y)
          if (q[y].size() - pos[y] > q[src].size() - pos[src]) src = y;
        if (pos[src] >= q[src].size()) break;
      }
      tasks.push_back(q[src][pos[src]++]);
      --left;
      if (left == 0) break;
    }
  }
}

static int ensure_zeros(svar_handle* h, int64_t n, hipStream_t st) {
  if (n <= h->zeros_elems) return SVAR_OK;
  if (h->zeros) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(h->zeros);
    auto it = std::find(h->allocs.begin(), h->allocs.end(), (void*)h->zeros);
    if (it != h->allocs.end()) h->allocs.erase(it);
  }
  h->zeros = nullptr;
  h->zeros_elems = 0;
  SVAR_TRY(dalloc(h->allocs, &h->zeros, (size_t)n));
  launch_fill(h->zeros, n, 0.0, st);
  SVAR_HIP(hipStreamSynchronize(st));
  h->zeros_elems = n;
  return SVAR_OK;
}

static std::string gemm_key(int dtype, const std::vector<GemmProb>& probs) {
  std::string k = dtype == DT_F64 ? "f64" : (dtype == DT_F32 ? "f32" : "bf16");
  for (auto& p : probs) k += "|" + std::to_string(p.n) + "x" + std::to_string(p.ncols);
  return k;
}

// tiled < 0: the autotuned choice for this shape if one is known, else the default
static int make_gemm_plan(svar_handle* h, std::vector<void*>& owner, std::vector<GemmProb>& probs,
                          int dtype, GemmPlanDev& g, hipStream_t st, int tiled = -1,
                          int target = 512) {
  std::vector<GemmTask> tasks;
  int64_t ws = 0;
  int maxct = 1;
  int64_t nmax = 1;
  for (auto& p : probs) nmax = std::max<int64_t>(nmax, p.n);
  SVAR_TRY(ensure_zeros(h, nmax, st));
  for (auto& p : probs) {
    p.dtype = dtype;
    p.zeros = h->zeros;
    if (p.ld <= 0) p.ld = p.n;
  }
  int maxcols = 1;
  for (auto& p : probs) maxcols = std::max(maxcols, p.ncols);
  g.key = gemm_key(dtype, probs);
  if (tiled < 0) {
    // default: the tiled kernel once the panel spans several 128-column groups (measured on
    // C2: k-split 93 us vs tiled 103 us at 65 columns, tiled ahead at 520)
    tiled = maxcols > 128 ? 1 : 0;
    auto it = h->tune.find(g.key);
    if (it != h->tune.end()) {
      tiled = it->second.first;
      target = it->second.second;
    }
  }
  if (maxcols < 32) tiled = 0;  // the tiled kernel needs two or more 16-column tiles
  g.tiled = tiled;
  g.target = target;
  g.direct = 1;
  const size_t esz = dtype == DT_F64 ? 8 : (dtype == DT_F32 ? 4 : 2);
  for (auto& p : probs)
    if ((p.ld & 3) != 0 || ((uintptr_t)p.C & (4 * esz - 1)) != 0) g.direct = 0;
  g.hprobs = probs;
  if (g.tiled)
    plan_gemm_tiled(probs, tasks, ws, maxct, target);
  else
    plan_gemm(probs, tasks, ws, maxct, target);
  g.nprob = (int)probs.size();
  g.ntask = (int)tasks.size();
  g.maxct = maxct;
  g.ws_elems = ws;
  g.dtype = dtype;
  g.reduce_probs.clear();
  g.max_reduce_elems = 0;
  for (int i = 0; i < (int)probs.size(); ++i)
    if (probs[i].splits > 1) {
      g.reduce_probs.push_back(i);
      g.max_reduce_elems = std::max(g.max_reduce_elems, (int64_t)probs[i].n * probs[i].ncols);
    }
  SVAR_TRY(upload(owner, &g.probs, probs.data(), probs.size(), st));
  SVAR_TRY(upload(owner, &g.tasks, tasks.data(), tasks.size(), st));
  if (!g.reduce_probs.empty())
    SVAR_TRY(upload(owner, &g.reduce_list, g.reduce_probs.data(), g.reduce_probs.size(), st));
  return SVAR_OK;
}

static int regrow(svar_handle* h, double** buf, int64_t* have, int64_t need) {
  if (need <= *have) return SVAR_OK;
  if (*buf) {
    (void)hipFree(*buf);
    auto it = std::find(h->allocs.begin(), h->allocs.end(), (void*)*buf);
    if (it != h->allocs.end()) h->allocs.erase(it);
  }
  *buf = nullptr;
  *have = 0;
  SVAR_TRY(dalloc(h->allocs, buf, (size_t)need));
  *have = need;
  return SVAR_OK;
}

// Y = C X for square set-up products (absolute pointers, column-major panels, ld = n)
static int gemm_abs(svar_handle* h, const double* C, int n, const double* X, double* Y, int ncols,
                    hipStream_t st) {
  GemmProb p{};
  p.C = C;
  p.n = n;
  p.ncols = ncols;
  p.per = ncols;
  p.X = {B_IN, 0, 0};
  p.Y = {B_OUT, 0, 0};
  p.Z = {-1, 0, 0};
  p.xi = n;
  p.yi = n;
  p.alpha0 = 1.0;
  std::vector<GemmProb> probs{p};
  std::vector<void*> tmp;
  GemmPlanDev g;
  int rc = make_gemm_plan(h, tmp, probs, DT_F64, g, st);
  if (rc == SVAR_OK) rc = regrow(h, &h->gemm_ws, &h->gemm_ws_elems, g.ws_elems);
  if (rc == SVAR_OK) {
    Bases b{};
    b.p[B_IN] = const_cast<double*>(X);
    b.p[B_OUT] = Y;
    launch_gemm(g, b, h->gemm_ws, nullptr, st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      set_error(std::string("set-up GEMM failed: ") + hipGetErrorString(e));
      rc = SVAR_E_HIP;
    }
  }
  free_all(tmp);
  return rc;
}

// out = A^{-1} for symmetric positive definite A by Newton-Schulz: X0 = I/||A||_inf (all
// eigenvalues of A X0 in (0, 1]), X <- X (2I - A X) until ||I - A X||_F stops shrinking.
// SVAR_E_NOTSPD when the residual grows (A has a non-positive eigenvalue).
static int inverse_spd(svar_handle* h, const double* A, int n, double* out, hipStream_t st,
                       const std::string& what) {
  std::vector<void*> tmp;
  double *T = nullptr, *alt = nullptr, *rows = nullptr, *part = nullptr;
  SVAR_TRY(dalloc(tmp, &T, (size_t)n * n));
  int rc = dalloc(tmp, &alt, (size_t)n * n);
  if (rc == SVAR_OK) rc = dalloc(tmp, &rows, (size_t)n);
  if (rc == SVAR_OK) rc = dalloc(tmp, &part, 1024);
  double anorm = 0.0;
  if (rc == SVAR_OK) {
    su_rowabs(A, n, rows, st);
    std::vector<double> hr(n);
    if (hipMemcpyAsync(hr.data(), rows, n * sizeof(double), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = SVAR_E_HIP;
    for (double v : hr) anorm = std::max(anorm, v);
    if (rc == SVAR_OK && (!(anorm > 0.0) || !std::isfinite(anorm))) {
      set_error(what + ": zero or non-finite matrix");
      rc = SVAR_E_NOTSPD;
    }
  }
  double* cur = out;
  if (rc == SVAR_OK) su_scaled_identity(cur, n, 1.0 / anorm, st);
  double first = -1.0;
  int extra = -1;
  for (int it = 0; rc == SVAR_OK && it < 300; ++it) {
    rc = gemm_abs(h, A, n, cur, T, n, st);  // T = A X
    if (rc != SVAR_OK) break;
    const int g = su_ns_residual(T, n, part, st);  // e = ||I - A X||_F ; T <- 2I - A X
    double e2 = 0.0;
    rc = host_sum(part, g, st, &e2);
    if (rc != SVAR_OK) break;
    const double e = std::sqrt(e2);
    if (first < 0) first = e;
    if (!std::isfinite(e) || e > 2.0 * first + 1.0) {
      set_error(what + ": not symmetric positive definite (Newton-Schulz diverged)");
      rc = SVAR_E_NOTSPD;
      break;
    }
    if (extra == 0) break;
    if (extra < 0 && e < 1e-4) extra = 2;  // quadratic phase: two more steps reach rounding
    if (it == 299) {
      set_error(what + ": Newton-Schulz inverse did not converge (matrix singular or too "
                       "ill-conditioned for an explicit inverse)");
      rc = SVAR_E_NOTSPD;
      break;
    }
    double* next = (cur == out) ? alt : out;
    rc = gemm_abs(h, cur, n, T, next, n, st);  // X <- X (2I - A X)
    cur = next;
    if (extra > 0) --extra;
  }
  if (rc == SVAR_OK) {
    if (cur != out) {
      if (hipMemcpyAsync(out, cur, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, st) !=
          hipSuccess)
        rc = SVAR_E_HIP;
    }
    su_symmetrize(out, n, st);
    if (hipStreamSynchronize(st) != hipSuccess) rc = SVAR_E_HIP;
  }
  free_all(tmp);
  return rc;
}

// Smallest eigenpair of SPD R given Minv = (a matrix whose dominant eigenvector is the wanted
// one, e.g. R^{-1}): repeated squaring M <- M^2 / ||M^2||_F converges to v v^T; v is the
// normalised largest row, lambda = v^T R v (Rayleigh quotient).
static int dominant_eigpair(svar_handle* h, const double* Minv, const double* R, int n,
                            double* lam, double* vdev, hipStream_t st) {
  std::vector<void*> tmp;
  double *M = nullptr, *M2 = nullptr, *part = nullptr, *rn = nullptr, *Rv = nullptr;
  SVAR_TRY(dalloc(tmp, &M, (size_t)n * n));
  int rc = dalloc(tmp, &M2, (size_t)n * n);
  if (rc == SVAR_OK) rc = dalloc(tmp, &part, 1024);
  if (rc == SVAR_OK) rc = dalloc(tmp, &rn, (size_t)n);
  if (rc == SVAR_OK) rc = dalloc(tmp, &Rv, (size_t)n);
  double f2 = 0.0;
  if (rc == SVAR_OK) {
    int g = su_sqdiff_part(Minv, nullptr, (int64_t)n * n, part, st);
    rc = host_sum(part, g, st, &f2);
  }
  if (rc == SVAR_OK) {
    su_copy_scale_shift(Minv, M, n, 1.0 / std::sqrt(f2), 0.0, st);
    for (int it = 0; it < 64 && rc == SVAR_OK; ++it) {
      rc = gemm_abs(h, M, n, M, M2, n, st);
      if (rc != SVAR_OK) break;
      double n2 = 0.0;
      int g = su_sqdiff_part(M2, nullptr, (int64_t)n * n, part, st);
      rc = host_sum(part, g, st, &n2);
      if (rc != SVAR_OK) break;
      if (!(n2 > 0.0) || !std::isfinite(n2)) {
        set_error("eigenvalue extraction: squaring underflowed");
        rc = SVAR_E_NOTSPD;
        break;
      }
      su_scale(M2, (int64_t)n * n, 1.0 / std::sqrt(n2), st);
      double d2 = 0.0;
      g = su_sqdiff_part(M2, M, (int64_t)n * n, part, st);
      rc = host_sum(part, g, st, &d2);
      std::swap(M, M2);
      if (d2 < 1e-28) break;
    }
  }
  if (rc == SVAR_OK) {
    su_rownorm2(M, n, rn, st);
    std::vector<double> hr(n);
    SVAR_HIP(hipMemcpyAsync(hr.data(), rn, n * sizeof(double), hipMemcpyDeviceToHost, st));
    SVAR_HIP(hipStreamSynchronize(st));
    const int row = (int)(std::max_element(hr.begin(), hr.end()) - hr.begin());
    su_row_scaled(M, n, row, 1.0 / std::sqrt(hr[row]), vdev, st);
    rc = gemm_abs(h, R, n, vdev, Rv, 1, st);
    double q = 0.0;
    if (rc == SVAR_OK) {
      int g = su_dot_part(vdev, Rv, n, part, st);
      rc = host_sum(part, g, st, &q);
    }
    *lam = q;
  }
  free_all(tmp);
  return rc;
}

// ------------------------------------------------------------------ window set-up
static int setup_model(svar_handle* h, WinDev& W, const svar_model_desc& md, hipStream_t st) {
  ModelDev M{};
  M.s = W.s;
  M.N = W.N;
  const int s = W.s;
  std::vector<int32_t> off;
  std::vector<double> wts;
  if (md.kind == SVAR_MODEL_BAND_DIRICHLET) {
    // a non-periodic band: the per-step model kernel with zero boundary values (no tap window,
    // so neither the windowed nor the fused sweep kernel, which wrap around the ring)
    M.kind = MK_BAND;
    M.nonperiodic = 1;
    if (md.ntaps < 1 || !md.offsets || !md.weights) return inval("band model needs taps");
    for (int t = 0; t < md.ntaps; ++t) {
      if (md.offsets[t] <= -s || md.offsets[t] >= s) return inval("band offset beyond the grid");
      off.push_back(md.offsets[t]);
      wts.push_back(md.weights[t]);
    }
    M.ntap = (int)off.size();
    std::vector<int32_t> offT(off.size());
    for (size_t t = 0; t < off.size(); ++t) offT[t] = -off[t];
    auto mm = std::minmax_element(off.begin(), off.end());
    M.omin = *mm.first;
    M.omax = *mm.second;
    M.ominT = -M.omax;
    M.omaxT = -M.omin;
    const int halo = M.omax - M.omin;
    if ((256 + halo) * 8 > 64 * 1024) return inval("band model too wide for the LDS tile");
    h->max_halo = std::max(h->max_halo, halo);
    int32_t *doff = nullptr, *doffT = nullptr;
    double* dw = nullptr;
    SVAR_TRY(upload(h->allocs, &doff, off.data(), off.size(), st));
    SVAR_TRY(upload(h->allocs, &doffT, offT.data(), offT.size(), st));
    SVAR_TRY(upload(h->allocs, &dw, wts.data(), wts.size(), st));
    M.off = doff;
    M.offT = doffT;
    M.w = dw;
    M.wT = dw;
    h->band_window = false;
  } else if (md.kind == SVAR_MODEL_CIRC_BAND || md.kind == SVAR_MODEL_PERIODIC_TRIDIAG_INV) {
    M.kind = MK_BAND;
    if (md.kind == SVAR_MODEL_CIRC_BAND) {
      if (md.ntaps < 1 || !md.offsets || !md.weights) return inval("band model needs taps");
      for (int t = 0; t < md.ntaps; ++t) {
        int o = md.offsets[t] % s;
        if (o > s / 2) o -= s;
        if (o < -(s - 1) / 2 - 1) o += s;
        off.push_back(o);
        wts.push_back(md.weights[t]);
      }
    } else {
      if (s < 3) return inval("periodic tridiagonal model needs s >= 3");
      if (!(std::fabs(md.tri_b) > std::fabs(md.tri_a) + std::fabs(md.tri_c)))
        return inval("periodic tridiagonal model must be strictly diagonally dominant");
      std::vector<void*> tmp;
      double *g = nullptr, *work = nullptr;
      SVAR_TRY(dalloc(tmp, &g, s));
      int rc = dalloc(tmp, &work, 3 * (size_t)s);
      std::vector<double> hg(s);
      if (rc == SVAR_OK) {
        su_tridiag_inv_col(md.tri_a, md.tri_b, md.tri_c, s, g, work, st);
        if (hipMemcpyAsync(hg.data(), g, s * sizeof(double), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
          rc = SVAR_E_HIP;
      }
      free_all(tmp);
      SVAR_TRY(rc);
      // (T^{-1} x)_j = sum_m g[(j - m) mod s] x_m: offset o = m - j has weight g[(-o) mod s].
      // Taps below 1e-20 of the largest are dropped (far under float64 resolution).
      double gmax = 0.0;
      for (double v : hg) gmax = std::max(gmax, std::fabs(v));
      for (int d = 0; d < s; ++d) {
        if (std::fabs(hg[d]) <= 1e-20 * gmax) continue;
        int o = -d;
        if (o < -(s / 2)) o += s;  // keep offsets in (-s/2, s/2]
        off.push_back(o);
        wts.push_back(hg[d]);
      }
    }
    M.ntap = (int)off.size();
    std::vector<int32_t> offT(off.size());
    for (size_t t = 0; t < off.size(); ++t) offT[t] = -off[t];
    auto mm = std::minmax_element(off.begin(), off.end());
    M.omin = *mm.first;
    M.omax = *mm.second;
    M.ominT = -M.omax;
    M.omaxT = -M.omin;
    const int halo = M.omax - M.omin;
    if ((256 + halo) * 8 > 64 * 1024) return inval("band model too wide for the LDS tile");
    h->max_halo = std::max(h->max_halo, halo);
    int32_t *doff = nullptr, *doffT = nullptr;
    double *dw = nullptr, *dwT = nullptr;
    SVAR_TRY(upload(h->allocs, &doff, off.data(), off.size(), st));
    SVAR_TRY(upload(h->allocs, &doffT, offT.data(), offT.size(), st));
    SVAR_TRY(upload(h->allocs, &dw, wts.data(), wts.size(), st));
    SVAR_TRY(upload(h->allocs, &dwT, wts.data(), wts.size(), st));
    M.off = doff;
    M.offT = doffT;
    M.w = dw;
    M.wT = dwT;
    // dense tap windows for the fused sweep kernel
    if (halo <= SWEEP_H && s >= SWEEP_H + 1) {
      std::vector<double> wdh(SWEEP_H + 1, 0.0), wdTh(SWEEP_H + 1, 0.0);
      for (size_t tp = 0; tp < off.size(); ++tp) {
        wdh[off[tp] - M.omin] += wts[tp];
        wdTh[offT[tp] - M.ominT] += wts[tp];
      }
      double *dwd = nullptr, *dwdT = nullptr;
      SVAR_TRY(upload(h->allocs, &dwd, wdh.data(), wdh.size(), st));
      SVAR_TRY(upload(h->allocs, &dwdT, wdTh.data(), wdTh.size(), st));
      M.wd = dwd;
      M.wdT = dwdT;
      M.wd0 = M.omin;
      M.wd0T = M.ominT;
    } else {
      h->band_window = false;
    }
  } else if (md.kind == SVAR_MODEL_DENSE) {
    M.kind = MK_DENSE;
    if (!md.dense) return inval("dense model needs N matrices");
    double* dm = nullptr;
    SVAR_TRY(dalloc(h->allocs, &dm, (size_t)W.N * s * s));
    for (int i = 0; i < W.N; ++i) {
      if (!md.dense[i]) return inval("dense model matrix missing");
      SVAR_HIP(hipMemcpyAsync(dm + (size_t)i * s * s, md.dense[i], (size_t)s * s * sizeof(double),
                              hipMemcpyHostToDevice, st));
    }
    M.dense = dm;
  } else if (md.kind == SVAR_MODEL_L96_TLM) {
    M.kind = MK_L96;
    if (!md.l96_traj || md.l96_nsteps < 1 || !(md.l96_dt > 0)) return inval("bad Lorenz-96 model");
    if (s < 4) return inval("Lorenz-96 tangent model needs s >= 4");
    if (md.l96_nsteps > 32) return inval("Lorenz-96 tangent model takes at most 32 RK4 steps per interval");
    h->l96_max_steps = std::max(h->l96_max_steps, md.l96_nsteps);
    double* tr = nullptr;
    SVAR_TRY(upload(h->allocs, &tr, md.l96_traj, (size_t)(W.N + 1) * s, st));
    M.traj = tr;
    M.F = md.l96_F;
    M.dt = md.l96_dt;
    M.nsteps = md.l96_nsteps;
  } else {
    return inval("unknown model kind");
  }
  W.model_kind = M.kind;
  W.model_id = (int)h->models.size();
  h->models.push_back(M);
  return SVAR_OK;
}

static int setup_window(svar_handle* h, WinDev& W, const svar_window_desc& d, hipStream_t st) {
  if (d.s < 1 || d.N < 0) return inval("window needs s >= 1 and N >= 0");
  W.s = d.s;
  W.N = d.N;
  W.nb = d.N + 1;
  const int s = W.s, nb = W.nb;
  if (!d.p || !d.dmats || !d.d_index || !d.d_scale || !d.rmats || !d.r_index)
    return inval("window descriptor has a NULL array");
  if (d.n_dmat < 1 || d.n_rmat < 1) return inval("need at least one D and one R matrix");
  W.p.assign(d.p, d.p + nb);
  W.poff.assign(nb + 1, 0);
  for (int i = 0; i < nb; ++i) {
    if (W.p[i] < 0) return inval("negative p_i");
    W.poff[i + 1] = W.poff[i] + W.p[i];
  }
  W.P = W.poff[nb];
  W.n = 2 * (int64_t)nb * s + W.P;
  // D
  W.d_index.assign(d.d_index, d.d_index + nb);
  W.d_scale.assign(d.d_scale, d.d_scale + nb);
  for (int i = 0; i < nb; ++i) {
    if (W.d_index[i] < 0 || W.d_index[i] >= d.n_dmat) return inval("d_index out of range");
    if (!(W.d_scale[i] > 0.0)) return inval("d_scale must be positive");
  }
  for (int m = 0; m < d.n_dmat; ++m) {
    double* p = nullptr;
    if (!d.dmats[m]) return inval("dmats entry is NULL");
    SVAR_TRY(upload(h->allocs, &p, d.dmats[m], (size_t)s * s, st));
    W.dmats.push_back(p);
  }
  SVAR_TRY(upload(h->allocs, &W.d_scale_dev, W.d_scale.data(), nb, st));
  std::vector<double> neg(nb);
  for (int i = 0; i < nb; ++i) neg[i] = -W.d_scale[i];
  SVAR_TRY(upload(h->allocs, &W.neg_d_scale_dev, neg.data(), nb, st));
  // R
  W.r_index.assign(d.r_index, d.r_index + nb);
  W.rmat_p.assign(d.n_rmat, -1);
  for (int i = 0; i < nb; ++i) {
    const int ri = W.r_index[i];
    if (ri < 0 || ri >= d.n_rmat) return inval("r_index out of range");
    if (W.rmat_p[ri] >= 0 && W.rmat_p[ri] != W.p[i])
      return inval("blocks sharing an R matrix must have the same p_i");
    W.rmat_p[ri] = W.p[i];
  }
  for (int m = 0; m < d.n_rmat; ++m) {
    double* p = nullptr;
    const int pm = std::max(W.rmat_p[m], 0);
    if (pm > 0 && !d.rmats[m]) return inval("rmats entry is NULL");
    if (pm > 0) {
      SVAR_TRY(upload(h->allocs, &p, d.rmats[m], (size_t)pm * pm, st));
    }
    W.rmats.push_back(p);
  }
  // H: ELL plus its transpose (CSR per block, index structure built here)
  if (d.h_width < 1) return inval("h_width must be >= 1");
  W.hw = d.h_width;
  const int64_t nent = (int64_t)W.P * W.hw;
  if (nent > 0 && (!d.h_cols || !d.h_vals)) return inval("H arrays are NULL");
  W.h_off.assign(nb, 0);
  for (int i = 0; i < nb; ++i) W.h_off[i] = (int64_t)W.poff[i] * W.hw;
  std::vector<int32_t> ptr((size_t)nb * (s + 1), 0), idx(nent);
  std::vector<double> val(nent);
  W.ht_ent_off.assign(nb, 0);
  for (int i = 0; i < nb; ++i) {
    int32_t* pp = ptr.data() + (size_t)i * (s + 1);
    const int64_t e0 = W.h_off[i];
    for (int64_t e = 0; e < (int64_t)W.p[i] * W.hw; ++e) {
      const int c = d.h_cols[e0 + e];
      if (c < 0 || c >= s) return inval("h_cols entry out of range");
      pp[c + 1]++;
    }
    for (int c = 0; c < s; ++c) pp[c + 1] += pp[c];
    std::vector<int32_t> fill(pp, pp + s);
    W.ht_ent_off[i] = e0;
    for (int64_t e = 0; e < (int64_t)W.p[i] * W.hw; ++e) {
      const int c = d.h_cols[e0 + e];
      const int64_t slot = e0 + fill[c]++;
      idx[slot] = (int32_t)(e / W.hw);  // observation row inside the block
      val[slot] = d.h_vals[e0 + e];
    }
  }
  SVAR_TRY(upload(h->allocs, &W.h_cols, d.h_cols, (size_t)nent, st));
  SVAR_TRY(upload(h->allocs, &W.h_vals, d.h_vals, (size_t)nent, st));
  SVAR_TRY(upload(h->allocs, &W.ht_ptr, ptr.data(), ptr.size(), st));
  SVAR_TRY(upload(h->allocs, &W.ht_idx, idx.data(), idx.size(), st));
  SVAR_TRY(upload(h->allocs, &W.ht_val, val.data(), val.size(), st));
  SVAR_TRY(setup_model(h, W, d.model, st));
  SVAR_HIP(hipStreamSynchronize(st));
  return SVAR_OK;
}

// Rhat^{-1} (§5, §6.1) and Dhat^{-1} (§6.1) on the GPU
// R_block (Alg. 3): groups of consecutive observation blocks kept whole.  normvec is formed on
// the device; the cut, split and combine rules run here; each group's inverse is formed by
// Newton-Schulz into one buffer (groups one after another, each n_g x n_g).
static int rblock_groups(const std::vector<int>& pvec, const std::vector<double>& normvec,
                         double tol, int maxsize, int numproc,
                         std::vector<std::pair<int, int>>& groups) {
  const int pn = (int)pvec.size();
  std::vector<int> pst(pn + 1, 0);
  for (int j = 0; j < pn; ++j) pst[j + 1] = pst[j] + pvec[j];
  std::vector<int> cuts{0};
  for (int j = 0; j + 1 < pn; ++j)
    if (normvec[j] < tol) cuts.push_back(pst[j + 1]);
  cuts.push_back(pst[pn]);
  groups.clear();
  for (size_t i = 0; i + 1 < cuts.size(); ++i) groups.push_back({cuts[i], cuts[i + 1]});
  auto size_of = [&](int i) { return groups[i].second - groups[i].first; };
  // a split cuts at the block boundary nearest the middle (the smaller one on a tie), a
  // one-block group at its middle row
  auto split = [&](int gi) {
    const int lo = groups[gi].first, hi = groups[gi].second;
    int best = -1;
    double bd = 0.0;
    for (int b : pst)
      if (b > lo && b < hi) {
        const double d = std::fabs(b - 0.5 * (lo + hi));
        if (best < 0 || d < bd) {
          best = b;
          bd = d;
        }
      }
    const int c = best >= 0 ? best : (lo + hi) / 2;
    groups[gi] = {lo, c};
    groups.insert(groups.begin() + gi + 1, std::make_pair(c, hi));
  };
  auto largest = [&]() {
    int bi = 0;
    for (int i = 1; i < (int)groups.size(); ++i)
      if (size_of(i) > size_of(bi)) bi = i;
    return bi;
  };
  if (maxsize > 0) {
    const int bi = largest();
    if (size_of(bi) > maxsize && size_of(bi) > 1) split(bi);
  }
  if (numproc > 0) {
    if ((int)groups.size() > numproc) {
      int bj = 0;
      for (int j = 1; j + 1 < (int)groups.size(); ++j)
        if (size_of(j) + size_of(j + 1) < size_of(bj) + size_of(bj + 1)) bj = j;
      groups[bj].second = groups[bj + 1].second;
      groups.erase(groups.begin() + bj + 1);
    } else if ((int)groups.size() < numproc - 2) {
      const int bi = largest();
      if (size_of(bi) > 1) split(bi);
    }
  }
  return SVAR_OK;
}

static int setup_rblock(svar_handle* h, WinDev& W, int m, hipStream_t st) {
  const int p = W.rmat_p[m];
  const std::vector<int>& pvec = h->rb_pvec;
  const int pn = (int)pvec.size();
  int tot = 0;
  for (int v : pvec) tot += v;
  if (tot != p) return inval("rb_pvec sums to " + std::to_string(tot) + " but R matrix " +
                             std::to_string(m) + " has " + std::to_string(p) + " rows");
  std::vector<int> pst(pn + 1, 0);
  for (int j = 0; j < pn; ++j) pst[j + 1] = pst[j] + pvec[j];
  std::vector<double> nv(std::max(pn - 1, 0));
  if (pn > 1) {
    std::vector<void*> tmp;
    int* dpst = nullptr;
    double* dnv = nullptr;
    SVAR_TRY(upload(tmp, &dpst, pst.data(), pst.size(), st));
    SVAR_TRY(dalloc(tmp, &dnv, nv.size()));
    su_superdiag_norms(W.rmats[m], p, dpst, pn - 1, dnv, st);
    SVAR_HIP(hipMemcpyAsync(nv.data(), dnv, nv.size() * sizeof(double), hipMemcpyDeviceToHost,
                            st));
    SVAR_HIP(hipStreamSynchronize(st));
    free_all(tmp);
  }
  std::vector<std::pair<int, int>> groups;
  SVAR_TRY(rblock_groups(pvec, nv, h->popts.rb_tol, h->popts.rb_maxsize, h->popts.rb_numproc,
                         groups));
  int64_t elems = 0;
  for (auto& g : groups) elems += (int64_t)(g.second - g.first) * (g.second - g.first);
  double* buf = nullptr;
  SVAR_TRY(dalloc(h->allocs, &buf, (size_t)elems));
  int64_t off = 0;
  for (auto& g : groups) {
    const int ng = g.second - g.first;
    std::vector<void*> tmp;
    double* blk = nullptr;
    SVAR_TRY(dalloc(tmp, &blk, (size_t)ng * ng));
    SVAR_HIP(hipMemcpy2DAsync(blk, (size_t)ng * sizeof(double),
                              W.rmats[m] + (int64_t)g.first * p + g.first,
                              (size_t)p * sizeof(double), (size_t)ng * sizeof(double), ng,
                              hipMemcpyDeviceToDevice, st));
    const int rc = inverse_spd(h, blk, ng, buf + off, st,
                               "R_block group at row " + std::to_string(g.first));
    SVAR_HIP(hipStreamSynchronize(st));
    free_all(tmp);
    SVAR_TRY(rc);
    W.rblk[m].push_back({(int64_t)g.first, (int64_t)g.second, off});
    off += (int64_t)ng * ng;
  }
  W.rhat_inv[m] = buf;
  W.rhat_inv_elems[m] = elems;
  return SVAR_OK;
}

static int setup_precond(svar_handle* h, WinDev& W, hipStream_t st) {
  const svar_prec_opts& po = h->popts;
  const int nr = (int)W.rmats.size();
  W.rhat_inv.assign(nr, nullptr);
  W.rhat_inv_elems.assign(nr, 0);
  W.rblk.assign(nr, {});
  W.rhat_dinv.assign(nr, nullptr);
  W.rr_gamma.assign(nr, std::numeric_limits<double>::quiet_NaN());
  W.me_T = W.rr_gamma;
  W.lam1 = W.rr_gamma;
  for (int m = 0; m < nr; ++m) {
    const int p = W.rmat_p[m];
    if (p <= 0) continue;
    const std::string what = "R matrix " + std::to_string(m);
    if (po.rhat == SVAR_RHAT_DIAG) {
      SVAR_TRY(dalloc(h->allocs, &W.rhat_dinv[m], (size_t)p));
      su_diag_inv(W.rmats[m], p, W.rhat_dinv[m], st);
      continue;
    }
    if (po.rhat == SVAR_RHAT_BLOCK) {
      SVAR_TRY(setup_rblock(h, W, m, st));
      continue;
    }
    double* Rinv = nullptr;
    SVAR_TRY(dalloc(h->allocs, &Rinv, (size_t)p * p));
    SVAR_TRY(inverse_spd(h, W.rmats[m], p, Rinv, st, what));
    W.rhat_inv_elems[m] = (int64_t)p * p;
    const bool need_l1 = (po.rhat == SVAR_RHAT_RR && po.rr_gamma < 0) || po.rhat == SVAR_RHAT_ME;
    std::vector<void*> tmp;
    double* v1 = nullptr;
    SVAR_TRY(dalloc(tmp, &v1, (size_t)p));
    double l1 = std::numeric_limits<double>::quiet_NaN();
    int rc = SVAR_OK;
    if (need_l1) rc = dominant_eigpair(h, Rinv, W.rmats[m], p, &l1, v1, st);
    W.lam1[m] = l1;
    if (rc == SVAR_OK && !(std::isnan(l1) || l1 > 0.0)) {
      set_error(what + ": smallest eigenvalue not positive");
      rc = SVAR_E_NOTSPD;
    }
    if (rc == SVAR_OK && po.rhat == SVAR_RHAT_RR) {
      // ridge regression (Alg. 1 with gamma chosen directly, §6.1): (R + gamma I)^{-1}
      const double gam = po.rr_gamma < 0 ? l1 : po.rr_gamma;
      W.rr_gamma[m] = gam;
      double* Rs = nullptr;
      rc = dalloc(tmp, &Rs, (size_t)p * p);
      if (rc == SVAR_OK) {
        su_copy_scale_shift(W.rmats[m], Rs, p, 1.0, gam, st);
        rc = inverse_spd(h, Rs, p, Rinv, st, what + " + gamma I");
      }
    } else if (rc == SVAR_OK && po.rhat == SVAR_RHAT_ME) {
      // minimum eigenvalue (Alg. 2, T = lambda_2 by default, §6.1).  Eigenvalues below T are
      // raised to T.  With T = lambda_2 only lambda_1 moves:
      //   R_ME^{-1} = R^{-1} + (1/T - 1/lambda_1) v_1 v_1^T.
      double T = po.me_T;
      if (T < 0) {
        // lambda_2: dominant eigenpair of R^{-1} - v1 v1^T / lambda_1
        double* Md = nullptr;
        double* v2 = nullptr;
        rc = dalloc(tmp, &Md, (size_t)p * p);
        if (rc == SVAR_OK) rc = dalloc(tmp, &v2, (size_t)p);
        if (rc == SVAR_OK) {
          su_copy_scale_shift(Rinv, Md, p, 1.0, 0.0, st);
          su_rank1(Md, p, v1, -1.0 / l1, st);
          rc = dominant_eigpair(h, Md, W.rmats[m], p, &T, v2, st);
        }
        if (p == 1) T = l1;
      } else if (po.me_T > l1 * (1.0 + 1e-12)) {
        // a threshold above lambda_2 would move more than one eigenvalue: build it fully
        rc = inval("R_ME with T above the second smallest eigenvalue is not supported");
      }
      W.me_T[m] = T;
      if (rc == SVAR_OK && T > l1) su_rank1(Rinv, p, v1, 1.0 / T - 1.0 / l1, st);
    }
    free_all(tmp);
    SVAR_TRY(rc);
    W.rhat_inv[m] = Rinv;
  }
  // per-block inverse diagonal for the DIAG kind
  if (po.rhat == SVAR_RHAT_DIAG && W.P > 0) {
    SVAR_TRY(dalloc(h->allocs, &W.rhat_dinv_blocks, (size_t)W.P));
    for (int i = 0; i < W.nb; ++i)
      if (W.p[i] > 0)
        SVAR_HIP(hipMemcpyAsync(W.rhat_dinv_blocks + W.poff[i], W.rhat_dinv[W.r_index[i]],
                                W.p[i] * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  // Dhat^{-1} = (d_scale_i D_{d_index i} + d_ridge I)^{-1}, one per distinct (matrix, scale)
  W.dhat_of_block.assign(W.nb, -1);
  if (po.type == SVAR_PREC_PD) {
    std::vector<std::pair<int, double>> keys;
    for (int i = 0; i < W.nb; ++i) {
      std::pair<int, double> key(W.d_index[i], W.d_scale[i]);
      auto it = std::find(keys.begin(), keys.end(), key);
      if (it == keys.end()) {
        keys.push_back(key);
        double *Dh = nullptr, *Dinv = nullptr;
        std::vector<void*> tmp;
        SVAR_TRY(dalloc(tmp, &Dh, (size_t)W.s * W.s));
        SVAR_TRY(dalloc(h->allocs, &Dinv, (size_t)W.s * W.s));
        su_copy_scale_shift(W.dmats[key.first], Dh, W.s, key.second, po.d_ridge, st);
        int rc = inverse_spd(h, Dh, W.s, Dinv, st, "Dhat block " + std::to_string(i));
        free_all(tmp);
        SVAR_TRY(rc);
        W.dhat_inv.push_back(Dinv);
        W.dhat_of_block[i] = (int)W.dhat_inv.size() - 1;
      } else {
        W.dhat_of_block[i] = (int)(it - keys.begin());
      }
    }
  }
  SVAR_HIP(hipStreamSynchronize(st));
  return SVAR_OK;
}

static int setup_lowprec(svar_handle* h, WinDev& W, hipStream_t st) {
  // float32 copies of D and R (inner operator of the mixed paths); bfloat16 copies of D,
  // Rhat^{-1} and Dhat^{-1} (preconditioner of MIXED_BF16P)
  auto conv = [&](const std::vector<double*>& src, std::vector<void*>& dst, int64_t elems_of,
                  bool bf16, const std::vector<int>* sizes) -> int {
    dst.assign(src.size(), nullptr);
    for (size_t m = 0; m < src.size(); ++m) {
      if (!src[m]) continue;
      const int64_t n = sizes ? (int64_t)(*sizes)[m] * (*sizes)[m] : elems_of;
      void* p = nullptr;
      if (bf16) {
        uint16_t* q = nullptr;
        SVAR_TRY(dalloc(h->allocs, &q, (size_t)n));
        p = q;
        su_to_bf16(src[m], p, n, st);
      } else {
        float* q = nullptr;
        SVAR_TRY(dalloc(h->allocs, &q, (size_t)n));
        p = q;
        su_to_f32(src[m], p, n, st);
      }
      dst[m] = p;
    }
    return SVAR_OK;
  };
  auto conv_n = [&](const std::vector<double*>& src, std::vector<void*>& dst,
                    const std::vector<int64_t>& elems, bool bf16) -> int {
    dst.assign(src.size(), nullptr);
    for (size_t m = 0; m < src.size(); ++m) {
      if (!src[m] || m >= elems.size() || elems[m] <= 0) continue;
      if (bf16) {
        uint16_t* q = nullptr;
        SVAR_TRY(dalloc(h->allocs, &q, (size_t)elems[m]));
        su_to_bf16(src[m], q, elems[m], st);
        dst[m] = q;
      } else {
        float* q = nullptr;
        SVAR_TRY(dalloc(h->allocs, &q, (size_t)elems[m]));
        su_to_f32(src[m], q, elems[m], st);
        dst[m] = q;
      }
    }
    return SVAR_OK;
  };
  // float32 copies of whole n x n matrices with rows padded to pad4(n) elements (zeros past
  // n), so that the GEMM kernels read every row with aligned 4-element loads
  auto conv_pad = [&](const std::vector<double*>& src, std::vector<void*>& dst, int n_all,
                      const std::vector<int>* sizes) -> int {
    dst.assign(src.size(), nullptr);
    for (size_t m = 0; m < src.size(); ++m) {
      if (!src[m]) continue;
      const int n = sizes ? (*sizes)[m] : n_all;
      if (n <= 0) continue;
      float* q = nullptr;
      SVAR_TRY(dalloc(h->allocs, &q, (size_t)n * pad4(n)));
      su_to_f32_pad(src[m], q, n, pad4(n), st);
      dst[m] = q;
    }
    return SVAR_OK;
  };
  const int64_t ss = (int64_t)W.s * W.s;
  SVAR_TRY(conv_pad(W.dmats, W.dmats_f32, W.s, nullptr));
  SVAR_TRY(conv_pad(W.rmats, W.rmats_f32, 0, &W.rmat_p));
  SVAR_TRY(conv(W.dmats, W.dmats_bf16, ss, true, nullptr));
  SVAR_TRY(conv_n(W.rhat_inv, W.rhat_inv_bf16, W.rhat_inv_elems, true));
  SVAR_TRY(conv(W.dhat_inv, W.dhat_inv_bf16, ss, true, nullptr));
  if (h->popts.rhat == SVAR_RHAT_BLOCK)  // group inverses stored one after another
    SVAR_TRY(conv_n(W.rhat_inv, W.rhat_inv_f32, W.rhat_inv_elems, false));
  else
    SVAR_TRY(conv_pad(W.rhat_inv, W.rhat_inv_f32, 0, &W.rmat_p));
  SVAR_TRY(conv_pad(W.dhat_inv, W.dhat_inv_f32, W.s, nullptr));
  SVAR_HIP(hipStreamSynchronize(st));
  return SVAR_OK;
}

// ------------------------------------------------------------------ layouts and builders
enum Space { SP_SADDLE = 0, SP_STATE = 1, SP_OBS = 2 };
enum Comp { C_ETA = 0, C_NU = 1, C_X = 2 };
struct VRef {
  int base;
  Space sp;
  int comp;
};

static int64_t sys_len(const WinDev& W, Space sp) {
  return sp == SP_SADDLE ? W.n : (sp == SP_STATE ? (int64_t)W.nb * W.s : (int64_t)W.P);
}
static int64_t win_base(const svar_handle* h, int w, int nrhs, Space sp) {
  int64_t o = 0;
  for (int i = 0; i < w; ++i) o += (int64_t)nrhs * sys_len(h->wins[i], sp);
  return o;
}
static int64_t comp_base(const WinDev& W, Space sp, int comp) {
  if (sp != SP_SADDLE) return 0;
  if (comp == C_ETA) return 0;
  if (comp == C_NU) return (int64_t)W.nb * W.s;
  return (int64_t)W.nb * W.s + W.P;
}
// offset of state block i (or obs block i) of system (w, r)
static Operand blk(const svar_handle* h, int w, int r, int nrhs, const VRef& v, int i) {
  const WinDev& W = h->wins[w];
  int64_t off = win_base(h, w, nrhs, v.sp) + r * sys_len(W, v.sp) + comp_base(W, v.sp, v.comp);
  off += (v.comp == C_NU) ? W.poff[i] : (int64_t)i * W.s;
  return Operand{v.base, 0, off};
}

struct Builder {
  svar_handle* h;
  int nrhs;
  hipStream_t st;
  Program* P;
  bool global_flag = false;  // every job retires on flag 0 only (all systems done)
};
// skip flag index (see Bases) of the jobs of system (w, r) and of window w's covariance products
static int sysflag(const Builder& B, int w, int r) {
  return B.global_flag ? 0 : 1 + w * B.nrhs + r;
}
static int winflag(const Builder& B, int w) {
  return B.global_flag ? 0 : 1 + (int)B.h->wins.size() * B.nrhs + w;
}

// the flat tile list of a job-table launch: lens[j] outputs of job j in tiles of JOB_TS
static int add_tiles(Builder& B, Launch& L, const std::vector<int>& lens) {
  std::vector<JTile> t;
  for (int j = 0; j < (int)lens.size(); ++j)
    for (int f = 0; f < lens[j]; f += JOB_TS) t.push_back(JTile{j, f});
  if (t.size() > (size_t)INT32_MAX) return SVAR_OK;  // keep the two-dimensional grid
  JTile* d = nullptr;
  SVAR_TRY(upload(B.h->allocs, &d, t.data(), t.size(), B.st));
  L.tiles = d;
  L.ntiles = (int)t.size();
  return SVAR_OK;
}

static int add_mjobs(Builder& B, std::vector<MJob> jobs[3]) {
  const LaunchKind kinds[3] = {LK_MSTEP_BAND, LK_MSTEP_DENSE, LK_MSTEP_L96};
  for (int k = 0; k < 3; ++k) {
    if (jobs[k].empty()) continue;
    Launch L;
    L.kind = kinds[k];
    L.njobs = (int)jobs[k].size();
    L.kclass = SVAR_KCLASS_MODEL;
    for (auto& j : jobs[k]) L.max_s = std::max(L.max_s, j.s);
    MJob* d = nullptr;
    SVAR_TRY(upload(B.h->allocs, &d, jobs[k].data(), jobs[k].size(), B.st));
    L.jobs = d;
    if (kinds[k] == LK_MSTEP_BAND) {
      std::vector<int> lens;
      for (auto& j : jobs[k]) lens.push_back(j.s);
      SVAR_TRY(add_tiles(B, L, lens));
    }
    B.P->launches.push_back(L);
  }
  return SVAR_OK;
}
static int kind_slot(const WinDev& W) {
  return W.model_kind == MK_BAND ? 0 : (W.model_kind == MK_DENSE ? 1 : 2);
}

// out = L in (trans = 0) or L^T in (trans = 1), eq. def:L
static int add_axpy_state(Builder& B, VRef in, VRef add, double beta, VRef out);

// out = L in (trans: L^T in), plus `add` when given (folded into the model kernels for band and
// dense models; Lorenz-96 windows take a separate vector pass)
static int add_L(Builder& B, VRef in, VRef out, int trans, VRef add = VRef{-1, SP_STATE, 0}) {
  if (add.base >= 0)
    for (const WinDev& W : B.h->wins)
      if (W.model_kind == MK_L96) {
        SVAR_TRY(add_L(B, in, out, trans));
        return add_axpy_state(B, out, add, 1.0, out);
      }
  std::vector<MJob> jobs[3];
  for (int w = 0; w < (int)B.h->wins.size(); ++w) {
    const WinDev& W = B.h->wins[w];
    for (int r = 0; r < B.nrhs; ++r)
      for (int i = 0; i < W.nb; ++i) {
        MJob J{};
        J.in = blk(B.h, w, r, B.nrhs, in, i);
        J.out = blk(B.h, w, r, B.nrhs, out, i);
        J.s = W.s;
        J.flag = sysflag(B, w, r);
        J.alpha = -1.0;
        J.trans = trans;
        if (add.base >= 0) {
          J.add = blk(B.h, w, r, B.nrhs, add, i);
          J.use_add = 1;
        }
        const bool has = trans ? (i < W.N) : (i >= 1);
        if (has) {
          J.model = W.model_id;
          J.mi = trans ? i + 1 : i;
          J.x = blk(B.h, w, r, B.nrhs, in, trans ? i + 1 : i - 1);
        } else {
          J.model = -1;
          J.x = J.in;
        }
        jobs[kind_slot(W)].push_back(J);
        if (has) B.P->cnt[trans ? 1 : 0] += 1;
      }
  }
  return add_mjobs(B, jobs);
}

// in-place sweep of L_M(k)^{-1} (trans = 0) or L_M(k)^{-T} (trans = 1) on vec (Lemma 1):
// step t updates position b + t (forward) / e - t (backward) of every segment.
static int add_copy_state(Builder& B, VRef in, VRef out, double alpha);

static bool sweep_fusable(const Builder& B, int k) {
  for (const WinDev& W : B.h->wins)
    if (W.model_kind != MK_BAND || W.s > SWEEP_MAXS || !B.h->models[W.model_id].wd) return false;
  return k > 1;
}

// vec = L_M(k)^{-1} (src - sub) (trans: L_M(k)^{-T}); src / sub NONE_REF: in place on vec
static int add_sweep(Builder& B, VRef vec, int trans, int k, VRef src = VRef{-1, SP_STATE, 0},
                     VRef sub = VRef{-1, SP_STATE, 0}) {
  if (B.h->popts.lhat == SVAR_LHAT_LI) {
    // L_I (§2.2): block running sums, one job per system, no model products
    std::vector<SJob> jobs;
    int ms = 0;
    for (int w = 0; w < (int)B.h->wins.size(); ++w) {
      const WinDev& W = B.h->wins[w];
      for (int r = 0; r < B.nrhs; ++r) {
        SJob J{};
        J.vec = blk(B.h, w, r, B.nrhs, vec, 0);
        J.src = src.base >= 0 ? blk(B.h, w, r, B.nrhs, src, 0) : Operand{-1, 0, 0};
        J.sub = sub.base >= 0 ? blk(B.h, w, r, B.nrhs, sub, 0) : Operand{-1, 0, 0};
        J.model = -1;
        J.trans = trans;
        J.s = W.s;
        J.len = W.nb;
        J.flag = sysflag(B, w, r);
        ms = std::max(ms, W.s);
        jobs.push_back(J);
      }
    }
    Launch L;
    L.kind = LK_PREFIX;
    L.njobs = (int)jobs.size();
    L.max_s = ms;
    L.kclass = SVAR_KCLASS_MODEL;
    SJob* d = nullptr;
    SVAR_TRY(upload(B.h->allocs, &d, jobs.data(), jobs.size(), B.st));
    L.jobs = d;
    B.P->launches.push_back(L);
    return SVAR_OK;
  }
  // band models with s <= SWEEP_MAXS: one fused launch, one workgroup per segment and rhs
  std::vector<SJob> fused;
  const bool outplace = src.base >= 0 || sub.base >= 0;
  if (outplace && !sweep_fusable(B, k)) {
    // the per-step path sweeps in place: form src - sub (or copy src) first
    if (sub.base >= 0)
      SVAR_TRY(add_axpy_state(B, src, sub, -1.0, vec));
    else
      SVAR_TRY(add_copy_state(B, src, vec, 1.0));
    return add_sweep(B, vec, trans, k);
  }
  if (sweep_fusable(B, k)) {
    int ms = 0;
    for (int w = 0; w < (int)B.h->wins.size(); ++w) {
      const WinDev& W = B.h->wins[w];
      for (int r = 0; r < B.nrhs; ++r)
        for (int b0 = 0; b0 <= W.N; b0 += k) {
          const int e0 = std::min(b0 + k - 1, W.N);
          if (e0 == b0 && !outplace) continue;
          SJob J{};
          J.src = src.base >= 0 ? blk(B.h, w, r, B.nrhs, src, b0) : Operand{-1, 0, 0};
          J.sub = sub.base >= 0 ? blk(B.h, w, r, B.nrhs, sub, b0) : Operand{-1, 0, 0};
          J.vec = blk(B.h, w, r, B.nrhs, vec, b0);
          J.model = W.model_id;
          J.flag = sysflag(B, w, r);
          J.trans = trans;
          J.s = W.s;
          J.len = e0 - b0 + 1;
          ms = std::max(ms, W.s);
          fused.push_back(J);
          B.P->cnt[trans ? 1 : 0] += e0 - b0;
        }
    }
    if (fused.empty()) return SVAR_OK;
    Launch L;
    L.kind = LK_SWEEP_BAND;
    L.njobs = (int)fused.size();
    L.max_s = ms;
    L.kclass = SVAR_KCLASS_MODEL;
    SJob* d = nullptr;
    SVAR_TRY(upload(B.h->allocs, &d, fused.data(), fused.size(), B.st));
    L.jobs = d;
    B.P->launches.push_back(L);
    return SVAR_OK;
  }
  for (int t = 1; t < k; ++t) {
    std::vector<MJob> jobs[3];
    for (int w = 0; w < (int)B.h->wins.size(); ++w) {
      const WinDev& W = B.h->wins[w];
      for (int r = 0; r < B.nrhs; ++r)
        for (int b0 = 0; b0 <= W.N; b0 += k) {
          const int e0 = std::min(b0 + k - 1, W.N);
          const int i = trans ? e0 - t : b0 + t;
          if (i < b0 || i > e0) continue;
          MJob J{};
          J.in = blk(B.h, w, r, B.nrhs, vec, i);
          J.out = J.in;
          J.flag = sysflag(B, w, r);
          J.x = blk(B.h, w, r, B.nrhs, vec, trans ? i + 1 : i - 1);
          J.model = W.model_id;
          J.mi = trans ? i + 1 : i;
          J.trans = trans;
          J.s = W.s;
          J.alpha = 1.0;
          jobs[kind_slot(W)].push_back(J);
          B.P->cnt[trans ? 1 : 0] += 1;
        }
    }
    SVAR_TRY(add_mjobs(B, jobs));
  }
  return SVAR_OK;
}

static int add_vjobs(Builder& B, std::vector<VJob>& jobs) {
  if (jobs.empty()) return SVAR_OK;
  Launch L;
  L.kind = LK_VEC;
  L.njobs = (int)jobs.size();
  int64_t ml = 0;
  for (auto& j : jobs) ml = std::max(ml, j.len);
  L.max_s = (int)std::min<int64_t>(ml, 1 << 30);
  VJob* d = nullptr;
  SVAR_TRY(upload(B.h->allocs, &d, jobs.data(), jobs.size(), B.st));
  L.jobs = d;
  B.P->launches.push_back(L);
  return SVAR_OK;
}

// out_state_component = alpha * in_state_component (whole state component of each system)
// out = in + beta * add over every system's state-sized component
static int add_axpy_state(Builder& B, VRef in, VRef add, double beta, VRef out) {
  std::vector<VJob> jobs;
  for (int w = 0; w < (int)B.h->wins.size(); ++w) {
    const WinDev& W = B.h->wins[w];
    for (int r = 0; r < B.nrhs; ++r) {
      VJob J{};
      J.in = blk(B.h, w, r, B.nrhs, in, 0);
      J.out = blk(B.h, w, r, B.nrhs, out, 0);
      J.add = blk(B.h, w, r, B.nrhs, add, 0);
      J.alpha = 1.0;
      J.beta = beta;
      J.flag = sysflag(B, w, r);
      J.len = (int64_t)W.nb * W.s;
      jobs.push_back(J);
    }
  }
  return add_vjobs(B, jobs);
}
static int add_copy_state(Builder& B, VRef in, VRef out, double alpha) {
  std::vector<VJob> jobs;
  for (int w = 0; w < (int)B.h->wins.size(); ++w) {
    const WinDev& W = B.h->wins[w];
    for (int r = 0; r < B.nrhs; ++r) {
      VJob J{};
      J.in = blk(B.h, w, r, B.nrhs, in, 0);
      J.out = blk(B.h, w, r, B.nrhs, out, 0);
      J.alpha = alpha;
      J.len = (int64_t)W.nb * W.s;
      J.flag = sysflag(B, w, r);
      jobs.push_back(J);
    }
  }
  return add_vjobs(B, jobs);
}
// In-place network correction of the state vector vec (every window and rhs): one sample per
// (system, block), 64-point tiles, activations in row chunks of bounded size.
static int add_net(Builder& B, VRef vec) {
  const int64_t ROW_CHUNK = (int64_t)1 << 24;
  const int64_t SUM_CHUNK = (int64_t)1 << 13;
  auto app = std::make_unique<NetApp>();
  app->base = vec.base;
  std::vector<NetChunk> ch;
  std::vector<int32_t> c0;
  std::vector<NetSample> smp;
  std::vector<NetTile> tiles, ftiles;
  int64_t rows = 0;
  int sys = 0;
  app->tile0.push_back(0);
  app->ftile0.push_back(0);
  app->row0.push_back(0);
  for (int w = 0; w < (int)B.h->wins.size(); ++w) {
    const WinDev& W = B.h->wins[w];
    const int64_t len = (int64_t)W.nb * W.s;
    const int tps = (W.s + NET_TILE - 1) / NET_TILE;
    const int ftps = (W.s + NET_FTILE - 1) / NET_FTILE;
    for (int r = 0; r < B.nrhs; ++r, ++sys) {
      const int64_t off = blk(B.h, w, r, B.nrhs, vec, 0).off;
      app->spans.push_back({off, off + len});
      c0.push_back((int)ch.size());
      for (int64_t e = 0; e < len; e += SUM_CHUNK) {
        NetChunk c{};
        c.sys = sys;
        c.e0 = off + e;
        c.e1 = off + std::min(len, e + SUM_CHUNK);
        ch.push_back(c);
      }
      // start a new row chunk when this system would overflow the current one
      if (rows - app->row0.back() + len > ROW_CHUNK && rows > app->row0.back()) {
        app->max_rows = std::max(app->max_rows, rows - app->row0.back());
        app->tile0.push_back((int)tiles.size());
        app->ftile0.push_back((int)ftiles.size());
        app->row0.push_back(rows);
      }
      for (int i = 0; i < W.nb; ++i) {
        NetSample S{};
        S.src = off;
        S.row0 = rows;
        S.s = W.s;
        S.nb = W.nb;
        S.blk = i;
        S.sys = sys;
        const int q = (int)smp.size();
        smp.push_back(S);
        for (int t = 0; t < tps; ++t) tiles.push_back(NetTile{q, t * NET_TILE});
        for (int t = 0; t < ftps; ++t) ftiles.push_back(NetTile{q, t * NET_FTILE});
        rows += W.s;
      }
    }
  }
  c0.push_back((int)ch.size());
  app->max_rows = std::max(app->max_rows, rows - app->row0.back());
  app->tile0.push_back((int)tiles.size());
  app->ftile0.push_back((int)ftiles.size());
  app->nsys = sys;
  app->nchunk = (int)ch.size();
  app->ntiles = (int)tiles.size();
  app->nftiles = (int)ftiles.size();
  auto& A = B.h->allocs;
  SVAR_TRY(upload(A, &app->chunks, ch.data(), ch.size(), B.st));
  SVAR_TRY(upload(A, &app->chunk0, c0.data(), c0.size(), B.st));
  SVAR_TRY(upload(A, &app->smp, smp.data(), smp.size(), B.st));
  SVAR_TRY(upload(A, &app->tiles, tiles.data(), tiles.size(), B.st));
  SVAR_TRY(upload(A, &app->ftiles, ftiles.data(), ftiles.size(), B.st));
  SVAR_TRY(dalloc(A, &app->part, ch.size()));
  SVAR_TRY(dalloc(A, &app->sigma, (size_t)sys));
  SVAR_TRY(dalloc(A, &app->inv_sigma, (size_t)sys));
  SVAR_HIP(hipStreamSynchronize(B.st));
  Launch L;
  L.kind = LK_NET;
  L.jobs = app.get();
  L.kclass = SVAR_KCLASS_NET;
  B.P->launches.push_back(L);
  B.h->netapps.push_back(std::move(app));
  return SVAR_OK;
}
static int add_copy_obs(Builder& B, VRef in, VRef out, bool diag_rhat) {
  std::vector<VJob> jobs;
  for (int w = 0; w < (int)B.h->wins.size(); ++w) {
    const WinDev& W = B.h->wins[w];
    if (W.P == 0) continue;
    for (int r = 0; r < B.nrhs; ++r) {
      VJob J{};
      J.in = blk(B.h, w, r, B.nrhs, in, 0);
      J.out = blk(B.h, w, r, B.nrhs, out, 0);
      J.alpha = 1.0;
      J.scale = diag_rhat ? W.rhat_dinv_blocks : nullptr;
      J.len = W.P;
      J.flag = sysflag(B, w, r);
      jobs.push_back(J);
    }
    if (diag_rhat) B.P->cnt[4] += (int64_t)W.nb * B.nrhs;
  }
  return add_vjobs(B, jobs);
}

static int add_gather(Builder& B, VRef x, VRef out) {
  std::vector<HJob> jobs;
  int mr = 0;
  for (int w = 0; w < (int)B.h->wins.size(); ++w) {
    const WinDev& W = B.h->wins[w];
    for (int r = 0; r < B.nrhs; ++r)
      for (int i = 0; i < W.nb; ++i) {
        if (W.p[i] == 0) continue;
        HJob J{};
        J.x = blk(B.h, w, r, B.nrhs, x, i);
        J.out = blk(B.h, w, r, B.nrhs, out, i);
        J.cols = W.h_cols + W.h_off[i];
        J.vals = W.h_vals + W.h_off[i];
        J.rows = W.p[i];
        J.width = W.hw;
        J.flag = sysflag(B, w, r);
        mr = std::max(mr, W.p[i]);
        jobs.push_back(J);
      }
  }
  if (jobs.empty()) return SVAR_OK;
  Launch L;
  L.kind = LK_GATHER;
  L.njobs = (int)jobs.size();
  L.max_s = mr;
  HJob* d = nullptr;
  SVAR_TRY(upload(B.h->allocs, &d, jobs.data(), jobs.size(), B.st));
  L.jobs = d;
  std::vector<int> lens;
  for (auto& j : jobs) lens.push_back(j.rows);
  SVAR_TRY(add_tiles(B, L, lens));
  B.P->launches.push_back(L);
  return SVAR_OK;
}

static int add_scatter(Builder& B, VRef y, VRef out) {
  std::vector<HTJob> jobs;
  int ms = 0;
  for (int w = 0; w < (int)B.h->wins.size(); ++w) {
    const WinDev& W = B.h->wins[w];
    for (int r = 0; r < B.nrhs; ++r)
      for (int i = 0; i < W.nb; ++i) {
        if (W.p[i] == 0) continue;
        HTJob J{};
        J.y = blk(B.h, w, r, B.nrhs, y, i);
        J.out = blk(B.h, w, r, B.nrhs, out, i);
        J.ptr = W.ht_ptr + (size_t)i * (W.s + 1);
        J.idx = W.ht_idx + W.ht_ent_off[i];
        J.val = W.ht_val + W.ht_ent_off[i];
        J.s = W.s;
        J.flag = sysflag(B, w, r);
        ms = std::max(ms, W.s);
        jobs.push_back(J);
      }
  }
  if (jobs.empty()) return SVAR_OK;
  Launch L;
  L.kind = LK_SCATTER;
  L.njobs = (int)jobs.size();
  L.max_s = ms;
  HTJob* d = nullptr;
  SVAR_TRY(upload(B.h->allocs, &d, jobs.data(), jobs.size(), B.st));
  L.jobs = d;
  std::vector<int> lens;
  for (auto& j : jobs) lens.push_back(j.s);
  SVAR_TRY(add_tiles(B, L, lens));
  B.P->launches.push_back(L);
  return SVAR_OK;
}

// which matrix family a covariance product uses
enum MatSel { MS_D = 0, MS_DHAT = 1, MS_R = 2, MS_RHAT = 3 };

static const void* mat_ptr(const WinDev& W, MatSel sel, int idx, int dtype) {
  switch (sel) {
    case MS_D:
      return dtype == DT_F64 ? (const void*)W.dmats[idx]
                             : (dtype == DT_F32 ? W.dmats_f32[idx] : W.dmats_bf16[idx]);
    case MS_DHAT:
      return dtype == DT_F64 ? (const void*)W.dhat_inv[idx]
                             : (dtype == DT_F32 ? W.dhat_inv_f32[idx] : W.dhat_inv_bf16[idx]);
    case MS_R:
      return dtype == DT_F64 ? (const void*)W.rmats[idx] : W.rmats_f32[idx];
    default:
      return dtype == DT_F64 ? (const void*)W.rhat_inv[idx]
                             : (dtype == DT_F32 ? W.rhat_inv_f32[idx] : W.rhat_inv_bf16[idx]);
  }
}

// Y = beta Z + alpha0 * alpha_i * (Mat_i X) for every block i; blocks sharing a matrix in a
// consecutive run become one GEMM over all their columns and right-hand sides.
static void add_cov(Builder& B, std::vector<GemmProb>& probs, MatSel sel, int dtype, VRef X,
                    VRef Y, VRef Z, bool scaled, double alpha0, double beta) {
  for (int w = 0; w < (int)B.h->wins.size(); ++w) {
    const WinDev& W = B.h->wins[w];
    const bool obs = (sel == MS_R || sel == MS_RHAT);
    auto key = [&](int i) {
      if (sel == MS_D) return W.d_index[i];
      if (sel == MS_DHAT) return W.dhat_of_block[i];
      return W.r_index[i];
    };
    int i = 0;
    while (i < W.nb) {
      int j = i + 1;
      while (j < W.nb && key(j) == key(i)) ++j;
      const int n = obs ? W.p[i] : W.s;
      if (n > 0) {
        GemmProb p{};
        p.C = mat_ptr(W, sel, key(i), dtype);
        p.n = n;
        // the float32 copies of whole matrices have rows padded to 4 elements (set-up)
        p.ld = (dtype == DT_F32 && !(sel == MS_RHAT && B.h->popts.rhat == SVAR_RHAT_BLOCK))
                   ? pad4(n)
                   : n;
        p.per = j - i;
        p.ncols = (j - i) * B.nrhs;
        p.X = blk(B.h, w, 0, B.nrhs, X, i);
        p.Y = blk(B.h, w, 0, B.nrhs, Y, i);
        p.Z = Z.base >= 0 ? blk(B.h, w, 0, B.nrhs, Z, i) : Operand{-1, 0, 0};
        p.xo = sys_len(W, X.sp);
        p.yo = sys_len(W, Y.sp);
        p.zo = Z.base >= 0 ? sys_len(W, Z.sp) : 0;
        p.xi = p.yi = p.zi = n;
        p.alpha = scaled ? W.d_scale_dev + i : nullptr;
        p.alpha0 = alpha0;
        p.beta = beta;
        p.flag = winflag(B, w);
        if (sel == MS_RHAT && B.h->popts.rhat == SVAR_RHAT_BLOCK) {
          // R_block: one product per group (rows [lo, hi) of every column; the columns keep
          // the block stride n)
          const size_t es = dtype == DT_F64 ? 8 : (dtype == DT_F32 ? 4 : 2);
          for (const auto& g : W.rblk[key(i)]) {
            GemmProb q = p;
            q.C = (const char*)p.C + g[2] * es;
            q.n = (int)(g[1] - g[0]);
            q.ld = q.n;
            q.X.off += g[0];
            q.Y.off += g[0];
            if (q.Z.base >= 0) q.Z.off += g[0];
            probs.push_back(q);
          }
        } else {
          probs.push_back(p);
        }
        const int cidx = sel == MS_D ? 2 : (sel == MS_R ? 3 : (sel == MS_RHAT ? 4 : 5));
        B.P->cnt[cidx] += (int64_t)(j - i) * B.nrhs;
      }
      i = j;
    }
  }
}

static int add_gemm(Builder& B, std::vector<GemmProb>& probs, int dtype) {
  if (probs.empty()) return SVAR_OK;
  Launch L;
  L.kind = LK_GEMM;
  L.kclass = SVAR_KCLASS_GEMM;
  SVAR_TRY(make_gemm_plan(B.h, B.h->allocs, probs, dtype, L.gemm, B.st));
  B.P->launches.push_back(L);
  return SVAR_OK;
}

static const VRef IN_SAD_ETA{B_IN, SP_SADDLE, C_ETA}, IN_SAD_NU{B_IN, SP_SADDLE, C_NU},
    IN_SAD_X{B_IN, SP_SADDLE, C_X};
static const VRef OUT_SAD_ETA{B_OUT, SP_SADDLE, C_ETA}, OUT_SAD_NU{B_OUT, SP_SADDLE, C_NU},
    OUT_SAD_X{B_OUT, SP_SADDLE, C_X};
static const VRef NONE_REF{-1, SP_SADDLE, 0};

static int64_t total_len(const svar_handle* h, int nrhs, Space sp) {
  return win_base(h, (int)h->wins.size(), nrhs, sp);
}

// Build the launch program of one operation.
static int build_program(svar_handle* h, int op, int nrhs, int prec, Program& P, hipStream_t st) {
  Builder B{h, nrhs, st, &P};
  const int k = h->popts.k;
  const int ptype = h->popts.type;
  const bool diag = h->popts.rhat == SVAR_RHAT_DIAG;
  // precisions: A's covariances in float32 for the mixed paths, P's covariances in bfloat16
  // for MIXED_BF16P (products with float32 accumulation)
  const VRef DZ1{B_AUX, SP_STATE, C_X};
  if (op == PROG_AD) {
    // A z for z = P_I u just formed by PROG_PD: c1 = L z3 + D z1 with D z1 from the buffer;
    // R in float64 (PV_F64) or float32 (PV_F32)
    const int dr = prec == PV_F32 ? DT_F32 : DT_F64;
    P.aux_elems = total_len(h, nrhs, SP_STATE);
    SVAR_TRY(add_L(B, IN_SAD_X, OUT_SAD_ETA, 0, DZ1));  // L z3 + D z1
    SVAR_TRY(add_L(B, IN_SAD_ETA, OUT_SAD_X, 1));
    SVAR_TRY(add_gather(B, IN_SAD_X, OUT_SAD_NU));
    SVAR_TRY(add_scatter(B, IN_SAD_NU, OUT_SAD_X));
    std::vector<GemmProb> probs;
    add_cov(B, probs, MS_R, dr, IN_SAD_NU, OUT_SAD_NU, OUT_SAD_NU, false, 1.0, 1.0);
    SVAR_TRY(add_gemm(B, probs, dr));
    return SVAR_OK;
  }
  if (op == PROG_PD) {
    // P_I with D z1 formed once and kept for PROG_AD: in float64, or in float32 for PV_F32ALL;
    // Rhat^{-1} in the given precision
    const int dt = prec == PV_BF16P ? DT_BF16
                                    : ((prec == PV_F32P || prec == PV_F32ALL) ? DT_F32 : DT_F64);
    const int dd = prec == PV_F32ALL ? DT_F32 : DT_F64;
    P.aux_elems = total_len(h, nrhs, SP_STATE);
    SVAR_TRY(add_sweep(B, OUT_SAD_ETA, 1, k, IN_SAD_X));  // c1 = Lhat^{-T} v3
    if (h->net) SVAR_TRY(add_net(B, OUT_SAD_ETA));
    std::vector<GemmProb> pd, pr;
    add_cov(B, pd, MS_D, dd, OUT_SAD_ETA, DZ1, NONE_REF, true, 1.0, 0.0);
    if (!diag) add_cov(B, dt == dd ? pd : pr, MS_RHAT, dt, IN_SAD_NU, OUT_SAD_NU, NONE_REF,
                       false, 1.0, 0.0);
    SVAR_TRY(add_gemm(B, pd, dd));
    if (!pr.empty()) SVAR_TRY(add_gemm(B, pr, dt));
    if (diag) SVAR_TRY(add_copy_obs(B, IN_SAD_NU, OUT_SAD_NU, true));
    SVAR_TRY(add_sweep(B, OUT_SAD_X, 0, k, IN_SAD_ETA, DZ1));  // Lhat^{-1} (v1 - D z1)
    return SVAR_OK;
  }
  if (op == PROG_A) {
    const int dt = prec == PV_F64 ? DT_F64 : DT_F32;
    // c1 = L v3 (+ D v1 below), c3 = L^T v1 (+ H^T v2 below), c2 = H v3 (+ R v2 below)
    SVAR_TRY(add_L(B, IN_SAD_X, OUT_SAD_ETA, 0));
    SVAR_TRY(add_L(B, IN_SAD_ETA, OUT_SAD_X, 1));
    SVAR_TRY(add_gather(B, IN_SAD_X, OUT_SAD_NU));
    SVAR_TRY(add_scatter(B, IN_SAD_NU, OUT_SAD_X));
    std::vector<GemmProb> probs;
    add_cov(B, probs, MS_D, dt, IN_SAD_ETA, OUT_SAD_ETA, OUT_SAD_ETA, true, 1.0, 1.0);
    add_cov(B, probs, MS_R, dt, IN_SAD_NU, OUT_SAD_NU, OUT_SAD_NU, false, 1.0, 1.0);
    SVAR_TRY(add_gemm(B, probs, dt));
    return SVAR_OK;
  }
  if (op == PROG_P) {
    const int dt = prec == PV_BF16P ? DT_BF16 : (prec == PV_F32P ? DT_F32 : DT_F64);
    if (ptype == SVAR_PREC_NONE) {
      std::vector<VJob> jobs;
      for (int w = 0; w < (int)h->wins.size(); ++w)
        for (int r = 0; r < nrhs; ++r) {
          VJob J{};
          J.in = Operand{B_IN, 0, win_base(h, w, nrhs, SP_SADDLE) + r * h->wins[w].n};
          J.out = Operand{B_OUT, 0, J.in.off};
          J.alpha = 1.0;
          J.len = h->wins[w].n;
          J.flag = sysflag(B, w, r);
          jobs.push_back(J);
        }
      return add_vjobs(B, jobs);
    }
    if (ptype == SVAR_PREC_PI) {
      // z1 = Lhat^{-T} v3 ; z3 = Lhat^{-1}(v1 - D z1) ; z2 = Rhat^{-1} v2   (§6.2)
      SVAR_TRY(add_copy_state(B, IN_SAD_X, OUT_SAD_ETA, 1.0));
      SVAR_TRY(add_sweep(B, OUT_SAD_ETA, 1, k));
      if (h->net) SVAR_TRY(add_net(B, OUT_SAD_ETA));
      std::vector<GemmProb> probs;
      add_cov(B, probs, MS_D, dt, OUT_SAD_ETA, OUT_SAD_X, IN_SAD_ETA, true, -1.0, 1.0);
      if (!diag) add_cov(B, probs, MS_RHAT, dt, IN_SAD_NU, OUT_SAD_NU, NONE_REF, false, 1.0, 0.0);
      SVAR_TRY(add_gemm(B, probs, dt));
      if (diag) SVAR_TRY(add_copy_obs(B, IN_SAD_NU, OUT_SAD_NU, true));
      SVAR_TRY(add_sweep(B, OUT_SAD_X, 0, k));
      return SVAR_OK;
    }
    // P_D: z1 = Dhat^{-1} v1, z2 = Rhat^{-1} v2, z3 = Lhat^{-1} D Lhat^{-T} v3   (§6.2)
    const VRef TMP_ST{B_TMP, SP_STATE, C_X};
    P.tmp_elems = std::max(P.tmp_elems, total_len(h, nrhs, SP_STATE));
    SVAR_TRY(add_copy_state(B, IN_SAD_X, TMP_ST, 1.0));
    SVAR_TRY(add_sweep(B, TMP_ST, 1, k));
    if (h->net) SVAR_TRY(add_net(B, TMP_ST));
    std::vector<GemmProb> probs;
    add_cov(B, probs, MS_D, dt, TMP_ST, OUT_SAD_X, NONE_REF, true, 1.0, 0.0);
    add_cov(B, probs, MS_DHAT, dt, IN_SAD_ETA, OUT_SAD_ETA, NONE_REF, false, 1.0, 0.0);
    if (!diag) add_cov(B, probs, MS_RHAT, dt, IN_SAD_NU, OUT_SAD_NU, NONE_REF, false, 1.0, 0.0);
    SVAR_TRY(add_gemm(B, probs, dt));
    if (diag) SVAR_TRY(add_copy_obs(B, IN_SAD_NU, OUT_SAD_NU, true));
    SVAR_TRY(add_sweep(B, OUT_SAD_X, 0, k));
    return SVAR_OK;
  }
  // component maps on state / obs vectors
  const VRef IS{B_IN, SP_STATE, C_X}, OS{B_OUT, SP_STATE, C_X};
  if (op == PROG_HARVEST) {
    B.global_flag = true;  // every system's slot is written while any system is active
    return add_copy_state(B, IN_SAD_X, OS, 1.0);
  }
  const VRef IO{B_IN, SP_OBS, C_NU}, OO{B_OUT, SP_OBS, C_NU};
  std::vector<GemmProb> probs;
  switch (op) {
    case SVAR_OP_L:
      return add_L(B, IS, OS, 0);
    case SVAR_OP_LT:
      return add_L(B, IS, OS, 1);
    case SVAR_OP_LHAT_INV:
      SVAR_TRY(add_copy_state(B, IS, OS, 1.0));
      return add_sweep(B, OS, 0, k);
    case SVAR_OP_LHAT_INVT:
      SVAR_TRY(add_copy_state(B, IS, OS, 1.0));
      return add_sweep(B, OS, 1, k);
    case SVAR_OP_D:
      add_cov(B, probs, MS_D, DT_F64, IS, OS, NONE_REF, true, 1.0, 0.0);
      return add_gemm(B, probs, DT_F64);
    case SVAR_OP_DHAT_INV:
      if (ptype != SVAR_PREC_PD) return inval("Dhat^{-1} exists only for the P_D preconditioner");
      add_cov(B, probs, MS_DHAT, DT_F64, IS, OS, NONE_REF, false, 1.0, 0.0);
      return add_gemm(B, probs, DT_F64);
    case SVAR_OP_R:
      add_cov(B, probs, MS_R, DT_F64, IO, OO, NONE_REF, false, 1.0, 0.0);
      return add_gemm(B, probs, DT_F64);
    case SVAR_OP_RHAT_INV:
      if (diag) return add_copy_obs(B, IO, OO, true);
      add_cov(B, probs, MS_RHAT, DT_F64, IO, OO, NONE_REF, false, 1.0, 0.0);
      return add_gemm(B, probs, DT_F64);
    case SVAR_OP_H:
      return add_gather(B, IS, OO);
    case SVAR_OP_HT:
      SVAR_TRY(add_copy_state(B, IS, OS, 0.0));  // zero the output
      return add_scatter(B, IO, OS);
    default:
      return inval("unknown operation code");
  }
}

// Host-side bounds check of every job table before a program is first used: each range a
// kernel will touch must lie inside the vector it addresses (lengths per base pointer).
struct Span {
  int base;
  int64_t lo, hi;  // [lo, hi)
};
static bool span_ok(const Span& s, const int64_t len[4]) {
  if (s.base < 0) return true;
  if (s.base > 3) return false;
  return s.lo >= 0 && s.hi <= len[s.base] && s.lo <= s.hi;
}
static int validate_program(const svar_handle* h, const Program& P, int64_t in_len,
                            int64_t out_len, hipStream_t st) {
  const int64_t len[4] = {in_len, out_len, P.tmp_elems, P.aux_elems};
  auto fail = [](const char* what) {
    set_error(std::string("internal layout error in ") + what);
    return SVAR_E_INVAL;
  };
  for (const Launch& L : P.launches) {
    std::vector<Span> spans;
    if (L.kind == LK_MSTEP_BAND || L.kind == LK_MSTEP_DENSE || L.kind == LK_MSTEP_L96) {
      std::vector<MJob> J(L.njobs);
      SVAR_HIP(hipMemcpyAsync(J.data(), L.jobs, J.size() * sizeof(MJob), hipMemcpyDeviceToHost, st));
      SVAR_HIP(hipStreamSynchronize(st));
      for (auto& j : J) {
        spans.push_back({j.in.base, j.in.off, j.in.off + j.s});
        spans.push_back({j.out.base, j.out.off, j.out.off + j.s});
        if (j.use_add) spans.push_back({j.add.base, j.add.off, j.add.off + j.s});
        if (j.model >= 0) {
          spans.push_back({j.x.base, j.x.off, j.x.off + j.s});
          if (j.model >= (int)h->models.size() || h->models[j.model].s != j.s) return fail("model");
          if (j.mi < 1 || j.mi > h->models[j.model].N) return fail("model index");
        }
      }
    } else if (L.kind == LK_SWEEP_BAND) {
      std::vector<SJob> J(L.njobs);
      SVAR_HIP(hipMemcpyAsync(J.data(), L.jobs, J.size() * sizeof(SJob), hipMemcpyDeviceToHost, st));
      SVAR_HIP(hipStreamSynchronize(st));
      for (auto& j : J) {
        spans.push_back({j.vec.base, j.vec.off, j.vec.off + (int64_t)j.len * j.s});
        spans.push_back({j.src.base, j.src.off, j.src.off + (int64_t)j.len * j.s});
        spans.push_back({j.sub.base, j.sub.off, j.sub.off + (int64_t)j.len * j.s});
        if (j.model < 0 || j.model >= (int)h->models.size() || h->models[j.model].kind != MK_BAND ||
            !h->models[j.model].wd || j.s > SWEEP_MAXS || j.len < 1)
          return fail("sweep job");
      }
    } else if (L.kind == LK_PREFIX) {
      std::vector<SJob> J(L.njobs);
      SVAR_HIP(hipMemcpyAsync(J.data(), L.jobs, J.size() * sizeof(SJob), hipMemcpyDeviceToHost, st));
      SVAR_HIP(hipStreamSynchronize(st));
      for (auto& j : J) {
        spans.push_back({j.vec.base, j.vec.off, j.vec.off + (int64_t)j.len * j.s});
        spans.push_back({j.src.base, j.src.off, j.src.off + (int64_t)j.len * j.s});
        spans.push_back({j.sub.base, j.sub.off, j.sub.off + (int64_t)j.len * j.s});
        if (j.len < 1 || j.s < 1 || j.s > L.max_s) return fail("running-sum job");
      }
    } else if (L.kind == LK_GATHER) {
      std::vector<HJob> J(L.njobs);
      SVAR_HIP(hipMemcpyAsync(J.data(), L.jobs, J.size() * sizeof(HJob), hipMemcpyDeviceToHost, st));
      SVAR_HIP(hipStreamSynchronize(st));
      for (auto& j : J) {
        spans.push_back({j.out.base, j.out.off, j.out.off + j.rows});
        spans.push_back({j.x.base, j.x.off, j.x.off + 1});  // columns validated at set-up (< s)
      }
    } else if (L.kind == LK_SCATTER) {
      std::vector<HTJob> J(L.njobs);
      SVAR_HIP(hipMemcpyAsync(J.data(), L.jobs, J.size() * sizeof(HTJob), hipMemcpyDeviceToHost, st));
      SVAR_HIP(hipStreamSynchronize(st));
      for (auto& j : J) {
        spans.push_back({j.out.base, j.out.off, j.out.off + j.s});
        spans.push_back({j.y.base, j.y.off, j.y.off + 1});
      }
    } else if (L.kind == LK_VEC) {
      std::vector<VJob> J(L.njobs);
      SVAR_HIP(hipMemcpyAsync(J.data(), L.jobs, J.size() * sizeof(VJob), hipMemcpyDeviceToHost, st));
      SVAR_HIP(hipStreamSynchronize(st));
      for (auto& j : J) {
        spans.push_back({j.out.base, j.out.off, j.out.off + j.len});
        if (j.scale || j.alpha != 0.0) spans.push_back({j.in.base, j.in.off, j.in.off + j.len});
        if (j.beta != 0.0) spans.push_back({j.add.base, j.add.off, j.add.off + j.len});
      }
    } else if (L.kind == LK_NET) {
      const NetApp* a = (const NetApp*)L.jobs;
      for (auto& sp : a->spans) spans.push_back({a->base, sp.first, sp.second});
      if (a->tile0.size() != a->row0.size() + 1 || a->tile0.back() != a->ntiles)
        return fail("network tiles");
    } else if (L.kind == LK_GEMM) {
      std::vector<GemmProb> G(L.gemm.nprob);
      SVAR_HIP(hipMemcpyAsync(G.data(), L.gemm.probs, G.size() * sizeof(GemmProb),
                              hipMemcpyDeviceToHost, st));
      SVAR_HIP(hipStreamSynchronize(st));
      for (auto& g : G) {
        if (g.ncols < 1 || g.per < 1 || g.n < 1 || g.ld < g.n) return fail("gemm shape");
        const int co = (g.ncols - 1) / g.per, ci = std::min(g.per - 1, g.ncols - 1);
        spans.push_back({g.X.base, g.X.off, g.X.off + co * g.xo + ci * g.xi + g.n});
        spans.push_back({g.Y.base, g.Y.off, g.Y.off + co * g.yo + ci * g.yi + g.n});
        if (g.Z.base >= 0) spans.push_back({g.Z.base, g.Z.off, g.Z.off + co * g.zo + ci * g.zi + g.n});
        if (g.xo < 0 || g.xi < 0 || g.yo < 0 || g.yi < 0) return fail("gemm stride");
      }
    }
    for (auto& s : spans)
      if (!span_ok(s, len)) return fail("job range");
  }
  return SVAR_OK;
}

static int64_t space_total(const svar_handle* h, int nrhs, int sp) {
  return total_len(h, nrhs, (Space)sp);
}
static void op_spaces(int op, int* in_sp, int* out_sp) {
  *in_sp = *out_sp = SP_STATE;
  if (op == PROG_A || op == PROG_P || op == PROG_AD || op == PROG_PD) {
    *in_sp = *out_sp = SP_SADDLE;
  } else if (op == PROG_HARVEST) {
    *in_sp = SP_SADDLE;
  } else if (op == SVAR_OP_R || op == SVAR_OP_RHAT_INV) {
    *in_sp = *out_sp = SP_OBS;
  } else if (op == SVAR_OP_H) {
    *out_sp = SP_OBS;
  } else if (op == SVAR_OP_HT) {
    *in_sp = SP_OBS;
  }
}

int get_program(svar_handle* h, int op, int nrhs, int prec, Program** out, hipStream_t st) {
  ProgKey key{op, nrhs, prec};
  auto it = h->progs.find(key);
  if (it == h->progs.end()) {
    Program P;
    SVAR_TRY(build_program(h, op, nrhs, prec, P, st));
    SVAR_HIP(hipStreamSynchronize(st));
    int isp, osp;
    op_spaces(op, &isp, &osp);
    SVAR_TRY(validate_program(h, P, space_total(h, nrhs, isp), space_total(h, nrhs, osp), st));
    it = h->progs.emplace(key, P).first;
  }
  *out = &it->second;
  return SVAR_OK;
}

// ------------------------------------------------------------------ timing
static void timer_begin(svar_handle* h, int kc, hipStream_t st, hipEvent_t* e0, hipEvent_t* e1) {
  if (h->parent) h = h->parent;  // a view records into its parent's timers
  *e0 = *e1 = nullptr;
  if (kc < 0 || kc >= SVAR_KCLASS_COUNT || !h->timers[kc].on) return;
  Timer& T = h->timers[kc];
  if (!T.pool.empty()) {
    *e0 = T.pool.back().first;
    *e1 = T.pool.back().second;
    T.pool.pop_back();
  } else {
    (void)hipEventCreate(e0);
    (void)hipEventCreate(e1);
  }
  (void)hipEventRecord(*e0, st);
}
static void timer_end(svar_handle* h, int kc, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (!e0) return;
  if (h->parent) h = h->parent;  // a view records into its parent's timers
  (void)hipEventRecord(e1, st);
  h->timers[kc].pending.emplace_back(e0, e1);
  h->timers[kc].launches += 1;
}
bool timing_any(const svar_handle* h) {
  if (h->parent) h = h->parent;
  for (const auto& T : h->timers)
    if (T.on) return true;
  return false;
}
void timed_begin(svar_handle* h, int kc, hipStream_t st, hipEvent_t* e0, hipEvent_t* e1) {
  timer_begin(h, kc, st, e0, e1);
}
void timed_end(svar_handle* h, int kc, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  timer_end(h, kc, st, e0, e1);
}

// ------------------------------------------------------------------ program execution
// Launches of a program with the given split-K workspace (no allocation, no check of the
// workspace sizes: the callers do that); timed: record the kernel-class timers.
static int exec_program(svar_handle* h, const Program& P, double* in, double* out,
                        hipStream_t st, const int* skip, const int* flags, double* gemm_ws,
                        bool timed);

int run_program(svar_handle* h, const Program& P, double* in, double* out, hipStream_t st,
                const int* skip, const int* flags) {
  if (P.tmp_elems > h->tmp_elems) SVAR_TRY(regrow(h, &h->tmp, &h->tmp_elems, P.tmp_elems));
  if (P.aux_elems > h->dz1_elems) SVAR_TRY(regrow(h, &h->dz1, &h->dz1_elems, P.aux_elems));
  for (const Launch& L : P.launches)
    if (L.kind == LK_GEMM && L.gemm.ws_elems > h->gemm_ws_elems)
      SVAR_TRY(regrow(h, &h->gemm_ws, &h->gemm_ws_elems, L.gemm.ws_elems));
  return exec_program(h, P, in, out, st, skip, flags, h->gemm_ws, true);
}

static int exec_program(svar_handle* h, const Program& P, double* in, double* out,
                        hipStream_t st, const int* skip, const int* flags, double* gemm_ws,
                        bool timed) {
  Bases b{};
  b.p[B_IN] = in;
  b.p[B_OUT] = out;
  b.p[B_TMP] = h->tmp;
  b.p[B_AUX] = P.aux_elems > 0 ? h->dz1 : nullptr;
  b.flags = flags;
  for (const Launch& L : P.launches) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) timer_begin(h, L.kclass, st, &e0, &e1);
    switch (L.kind) {
      case LK_MSTEP_BAND:
        launch_mstep_band((const MJob*)L.jobs, L.njobs, L.max_s, h->max_halo, h->models_dev, b,
                          skip, st, h->band_window, L.tiles, L.ntiles);
        break;
      case LK_MSTEP_DENSE:
        launch_mstep_dense((const MJob*)L.jobs, L.njobs, L.max_s, h->models_dev, b, skip, st);
        break;
      case LK_SWEEP_BAND:
        launch_sweep_band((const SJob*)L.jobs, L.njobs, L.max_s, h->models_dev, b, skip, st);
        break;
      case LK_PREFIX:
        launch_prefix((const SJob*)L.jobs, L.njobs, L.max_s, b, skip, st);
        break;
      case LK_MSTEP_L96:
        launch_mstep_l96((const MJob*)L.jobs, L.njobs, L.max_s, h->l96_max_steps, h->models_dev,
                         b, skip, st);
        break;
      case LK_GATHER:
        launch_gather((const HJob*)L.jobs, L.njobs, L.max_s, b, skip, st, L.tiles, L.ntiles);
        break;
      case LK_SCATTER:
        launch_scatter((const HTJob*)L.jobs, L.njobs, L.max_s, b, skip, st, L.tiles, L.ntiles);
        break;
      case LK_VEC:
        launch_vec((const VJob*)L.jobs, L.njobs, L.max_s, b, skip, st);
        break;
      case LK_GEMM:
        launch_gemm(L.gemm, b, gemm_ws, skip, st);
        break;
      case LK_NET: {
        const NetApp* a = (const NetApp*)L.jobs;
        SVAR_TRY(run_net(h, *a, b.p[a->base], skip, st));
        break;
      }
    }
    if (timed) timer_end(h, L.kclass, st, e0, e1);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
    return SVAR_E_HIP;
  }
  return SVAR_OK;
}

int64_t handle_total(const svar_handle* h, int nrhs) { return total_len(h, nrhs, SP_SADDLE); }
// ------------------------------------------------------------------ GEMM autotuning
struct TuneEntry {
  std::string key;
  int tiled, target;
  double us, default_us;
};

static void pv_of(int precision, int* pv_a, int* pv_p) {
  *pv_a = prec_a64(precision) ? PV_F64 : PV_F32;
  *pv_p = prec_pv_p(precision);
}

// Time each candidate plan of every covariance-product launch of the A and P programs for
// nrhs right-hand sides (one warm-up and five timed launches on zero-filled scratch vectors);
// keep the fastest per shape key.
static int autotune(svar_handle* h, int nrhs, int precision, std::vector<TuneEntry>& out,
                    hipStream_t st) {
  int pv_a, pv_p;
  pv_of(precision, &pv_a, &pv_p);
  Program *PA = nullptr, *PP = nullptr, *PAD = nullptr, *PPD = nullptr;
  SVAR_TRY(get_program(h, PROG_A, nrhs, pv_a, &PA, st));
  SVAR_TRY(get_program(h, PROG_P, nrhs, pv_p, &PP, st));
  std::vector<const Program*> progs = {PA, PP};
  if (h->popts.type == SVAR_PREC_PI && pv_a == PV_F64) {  // the solver's P_I / A pair
    SVAR_TRY(get_program(h, PROG_AD, nrhs, PV_F64, &PAD, st));
    SVAR_TRY(get_program(h, PROG_PD, nrhs, pv_p, &PPD, st));
    progs.push_back(PAD);
    progs.push_back(PPD);
    if (PPD->aux_elems > h->dz1_elems) SVAR_TRY(regrow(h, &h->dz1, &h->dz1_elems, PPD->aux_elems));
  }
  const int64_t len = total_len(h, nrhs, SP_SADDLE);
  std::vector<void*> tmp;
  double *vin = nullptr, *vout = nullptr;
  SVAR_TRY(dalloc(tmp, &vin, (size_t)len));
  int rc = dalloc(tmp, &vout, (size_t)len);
  if (rc == SVAR_OK) {
    launch_fill(vin, len, 0.0, st);
    launch_fill(vout, len, 0.0, st);
  }
  const int64_t tmp_need = std::max(PA->tmp_elems, PP->tmp_elems);
  if (rc == SVAR_OK && tmp_need > h->tmp_elems) rc = regrow(h, &h->tmp, &h->tmp_elems, tmp_need);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (rc == SVAR_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = inval("event creation failed");
  std::vector<GemmPlanDev> seen;
  for (const Program* P : progs) {
    for (const Launch& L : P->launches) {
      if (rc != SVAR_OK) break;
      if (L.kind != LK_GEMM) continue;
      if (h->tune.count(L.gemm.key) || std::any_of(out.begin(), out.end(), [&](const TuneEntry& e) {
            return e.key == L.gemm.key;
          }))
        continue;
      int maxcols = 1;
      for (auto& p : L.gemm.hprobs) maxcols = std::max(maxcols, p.ncols);
      std::vector<std::pair<int, int>> cands = {{0, 512}, {0, 1024}, {0, 2048}};
      if (maxcols >= 32) cands.insert(cands.end(), {{1, 256}, {1, 512}, {1, 768}, {1, 1024}});
      TuneEntry best{L.gemm.key, -1, 0, 1e30, 0.0};
      for (auto& c : cands) {
        std::vector<void*> owner;
        std::vector<GemmProb> probs = L.gemm.hprobs;
        GemmPlanDev g;
        rc = make_gemm_plan(h, owner, probs, L.gemm.dtype, g, st, c.first, c.second);
        if (rc == SVAR_OK && g.ws_elems > h->gemm_ws_elems)
          rc = regrow(h, &h->gemm_ws, &h->gemm_ws_elems, g.ws_elems);
        if (rc == SVAR_OK) {
          Bases b{};
          b.p[B_IN] = vin;
          b.p[B_OUT] = vout;
          b.p[B_TMP] = h->tmp;
          b.p[B_AUX] = h->dz1;  // written by the P_I program's D z1 product
          launch_gemm(g, b, h->gemm_ws, nullptr, st);
          (void)hipEventRecord(e0, st);
          for (int r = 0; r < 5; ++r) launch_gemm(g, b, h->gemm_ws, nullptr, st);
          (void)hipEventRecord(e1, st);
          if (hipEventSynchronize(e1) != hipSuccess) rc = inval("autotune launch failed");
          float ms = 0.0f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          const double us = 1e3 * ms / 5.0;
          const bool is_default = c.first == ((maxcols > 128) ? 1 : 0) && c.second == 512;
          if (is_default) best.default_us = us;
          if (us < best.us) {
            best.us = us;
            best.tiled = c.first;
            best.target = c.second;
          }
        }
        (void)hipStreamSynchronize(st);
        free_all(owner);
        if (rc != SVAR_OK) break;
      }
      if (rc == SVAR_OK && best.tiled >= 0) out.push_back(best);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  free_all(tmp);
  return rc;
}

static void drop_programs(svar_handle* h) {
  h->progs.clear();  // rebuilt on next use with the tuned plans
  h->prog_gen += 1;
}

int64_t state_total(const svar_handle* h, int nrhs) { return total_len(h, nrhs, SP_STATE); }

}  // namespace svar

// ====================================================================== C ABI
using namespace svar;

// ------------------------------------------------------------------ allocation-free A v
// The split-K partial sums of svar_apply_A_noalloc live in this file-scope device array (one
// copy per GPU, held until the process ends).  Host code never passes the array's name to a
// kernel: svar_create looks up its device address once per device (with that device current)
// and the entry point uses that address.
#define SVAR_NOALLOC_SCRATCH_ELEMS ((int64_t)1 << 23)  // 8 Mi doubles = 64 MiB per GPU
static __device__ __align__(256) double scratch[SVAR_NOALLOC_SCRATCH_ELEMS];
static std::mutex g_scratch_mu;
static constexpr int SCRATCH_MAX_DEV = 64;
static double* g_scratch_dev[SCRATCH_MAX_DEV] = {};

// device address of `scratch` on device dev (the current device), looked up on first use
static int scratch_setup(int dev) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEV) return inval("device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev]) return SVAR_OK;
  void* p = nullptr;
  SVAR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return inval("no device address for the scratch array");
  g_scratch_dev[dev] = (double*)p;
  return SVAR_OK;
}

extern "C" {

const char* svar_last_error(void) { return g_err.c_str(); }

int svar_autotune(svar_handle* h, int32_t nrhs, int32_t precision, const char* cache_path,
                  void* stream) {
  if (!h || nrhs < 1) return inval("bad arguments");
  if (!prec_valid(precision)) return inval("bad precision");
  hipStream_t st = (hipStream_t)stream;
  std::vector<TuneEntry> found;
  SVAR_TRY(autotune(h, nrhs, precision, found, st));
  for (auto& e : found) h->tune[e.key] = {e.tiled, e.target};
  if (!found.empty()) drop_programs(h);
  if (cache_path) {
    // merge with an existing cache: entries of this run replace those of the same key
    std::map<std::string, std::string> lines;
    if (FILE* f = std::fopen(cache_path, "r")) {
      char buf[1024];
      while (std::fgets(buf, sizeof(buf), f)) {
        std::string s(buf);
        const size_t a = s.find("\"key\": \"");
        if (a == std::string::npos) continue;
        const size_t b = s.find('"', a + 8);
        if (b == std::string::npos) continue;
        while (!s.empty() && (s.back() == '\n' || s.back() == ',')) s.pop_back();
        lines[s.substr(a + 8, b - a - 8)] = s;
      }
      std::fclose(f);
    }
    for (auto& e : found) {
      char buf[512];
      std::snprintf(buf, sizeof(buf),
                    "  {\"key\": \"%s\", \"tiled\": %d, \"target\": %d, \"us\": %.2f, "
                    "\"default_us\": %.2f}",
                    e.key.c_str(), e.tiled, e.target, e.us, e.default_us);
      lines[e.key] = buf;
    }
    FILE* f = std::fopen(cache_path, "w");
    if (!f) return inval(std::string("cannot write ") + cache_path);
    std::fprintf(f, "{\"version\": 1, \"entries\": [\n");
    size_t i = 0;
    for (auto& kv : lines)
      std::fprintf(f, "%s%s\n", kv.second.c_str(), ++i < lines.size() ? "," : "");
    std::fprintf(f, "]}\n");
    std::fclose(f);
  }
  return SVAR_OK;
}

int svar_autotune_load(svar_handle* h, const char* cache_path) {
  if (!h || !cache_path) return inval("bad arguments");
  FILE* f = std::fopen(cache_path, "r");
  if (!f) return inval(std::string("cannot read ") + cache_path);
  char buf[1024];
  int n = 0;
  while (std::fgets(buf, sizeof(buf), f)) {
    std::string s(buf);
    const size_t a = s.find("\"key\": \"");
    if (a == std::string::npos) continue;
    const size_t b = s.find('"', a + 8);
    const size_t ti = s.find("\"tiled\": "), ta = s.find("\"target\": ");
    if (b == std::string::npos || ti == std::string::npos || ta == std::string::npos) continue;
    const int tiled = std::atoi(s.c_str() + ti + 9);
    const int target = std::atoi(s.c_str() + ta + 10);
    if ((tiled != 0 && tiled != 1) || target < 1 || target > (1 << 20)) continue;
    h->tune[s.substr(a + 8, b - a - 8)] = {tiled, target};
    ++n;
  }
  std::fclose(f);
  if (n > 0) drop_programs(h);
  return SVAR_OK;
}

int svar_create(const svar_window_desc* windows, int32_t nwin, const svar_prec_opts* popts,
                svar_handle** out, void* stream) {
  if (!out) return inval("out is NULL");
  *out = nullptr;
  if (!windows || nwin < 1) return inval("need at least one window");
  if (!popts) return inval("popts is NULL");
  if (popts->type < SVAR_PREC_NONE || popts->type > SVAR_PREC_PI) return inval("bad prec type");
  if (popts->rhat < SVAR_RHAT_DIAG || popts->rhat > SVAR_RHAT_BLOCK) return inval("bad rhat kind");
  if (popts->type == SVAR_PREC_PD && !(popts->d_ridge >= 0.0)) return inval("bad d_ridge");
  if (popts->lhat != SVAR_LHAT_LM && popts->lhat != SVAR_LHAT_LI) return inval("bad lhat kind");
  hipStream_t st = (hipStream_t)stream;
  if (popts->rhat == SVAR_RHAT_BLOCK) {
    if (!popts->rb_pvec || popts->rb_npvec < 1) return inval("R_block needs rb_pvec");
    for (int j = 0; j < popts->rb_npvec; ++j)
      if (popts->rb_pvec[j] < 1) return inval("rb_pvec entries must be >= 1");
  }
  svar_handle* h = new svar_handle();
  h->popts = *popts;
  if (popts->rhat == SVAR_RHAT_BLOCK)
    h->rb_pvec.assign(popts->rb_pvec, popts->rb_pvec + popts->rb_npvec);
  h->popts.rb_pvec = nullptr;
  int rc = SVAR_OK;
  if (hipGetDevice(&h->device) != hipSuccess) rc = inval("no HIP device");
  if (rc == SVAR_OK) rc = scratch_setup(h->device);  // svar_apply_A_noalloc's scratch
  h->wins.resize(nwin);
  // the zero buffer that GEMM plans read past matrix edges is sized once for the largest
  // order (later growth would leave earlier plans pointing at a freed buffer)
  if (rc == SVAR_OK) {
    int64_t nmax = 1;
    for (int w = 0; w < nwin; ++w) {
      nmax = std::max<int64_t>(nmax, windows[w].s);
      if (windows[w].p && windows[w].N >= 0)
        for (int i = 0; i <= windows[w].N; ++i) nmax = std::max<int64_t>(nmax, windows[w].p[i]);
    }
    rc = ensure_zeros(h, nmax, st);
  }
  for (int w = 0; rc == SVAR_OK && w < nwin; ++w) {
    const int k = popts->k;
    if (k < 1 || k > windows[w].N + 1) rc = inval("k must satisfy 1 <= k <= N+1 (Definition 1)");
    if (rc == SVAR_OK) rc = setup_window(h, h->wins[w], windows[w], st);
    if (rc == SVAR_OK && popts->type != SVAR_PREC_NONE) rc = setup_precond(h, h->wins[w], st);
    if (rc == SVAR_OK) rc = setup_lowprec(h, h->wins[w], st);
  }
  if (rc == SVAR_OK) rc = upload(h->allocs, &h->models_dev, h->models.data(), h->models.size(), st);
  if (rc == SVAR_OK && hipStreamSynchronize(st) != hipSuccess) rc = inval("set-up sync failed");
  if (rc != SVAR_OK) {
    svar_destroy(h);
    return rc;
  }
  *out = h;
  return SVAR_OK;
}

int64_t svar_system_size(const svar_handle* h, int32_t w) {
  if (!h || w < 0 || w >= (int)h->wins.size()) return -1;
  return h->wins[w].n;
}

int svar_offsets(const svar_handle* h, int32_t nrhs, int64_t* off) {
  if (!h || !off || nrhs < 1) return inval("bad arguments");
  for (int w = 0; w <= (int)h->wins.size(); ++w) off[w] = win_base(h, w, nrhs, SP_SADDLE);
  return SVAR_OK;
}

int svar_apply_A_noalloc(svar_handle* h, int32_t nrhs, const double* v, double* y, void* stream) {
  if (!h || !v || !y || nrhs < 1) return inval("bad arguments");
  double* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (h->device >= 0 && h->device < SCRATCH_MAX_DEV) ws = g_scratch_dev[h->device];
  }
  if (!ws) return inval("scratch address of the handle's device was not set up");
  auto it = h->progs.find(ProgKey{PROG_A, nrhs, PV_F64});
  if (it == h->progs.end())
    return inval("no launch program for this nrhs yet: call svar_apply_A once with the same "
                 "nrhs first (this entry point builds nothing and allocates nothing)");
  const Program& P = it->second;
  if (P.tmp_elems > 0 || P.aux_elems > 0) return inval("program needs handle workspaces");
  for (const Launch& L : P.launches) {
    if (L.kind == LK_NET) return inval("program holds a network application");
    if (L.kind == LK_GEMM && L.gemm.ws_elems > SVAR_NOALLOC_SCRATCH_ELEMS)
      return inval("split-K partials of " + std::to_string(L.gemm.ws_elems) +
                   " doubles exceed the scratch array of " +
                   std::to_string(SVAR_NOALLOC_SCRATCH_ELEMS) + " doubles");
  }
  return exec_program(h, P, const_cast<double*>(v), y, (hipStream_t)stream, nullptr, nullptr,
                      ws, false);
}

int svar_apply_A(svar_handle* h, int32_t nrhs, const double* v, double* y, void* stream) {
  if (!h || !v || !y || nrhs < 1) return inval("bad arguments");
  Program* P = nullptr;
  hipStream_t st = (hipStream_t)stream;
  SVAR_TRY(get_program(h, PROG_A, nrhs, PV_F64, &P, st));
  return run_program(h, *P, const_cast<double*>(v), y, st, nullptr);
}

int svar_apply_P(svar_handle* h, int32_t nrhs, const double* v, double* z, void* stream) {
  if (!h || !v || !z || nrhs < 1) return inval("bad arguments");
  Program* P = nullptr;
  hipStream_t st = (hipStream_t)stream;
  SVAR_TRY(get_program(h, PROG_P, nrhs, PV_F64, &P, st));
  h->net_off = nullptr;  // outside a solve the correction always applies
  return run_program(h, *P, const_cast<double*>(v), z, st, nullptr);
}

int svar_apply_A_prec(svar_handle* h, int32_t precision, int32_t nrhs, const double* v, double* y,
                      void* stream) {
  if (!h || !v || !y || nrhs < 1) return inval("bad arguments");
  if (!prec_valid(precision)) return inval("bad precision");
  Program* P = nullptr;
  hipStream_t st = (hipStream_t)stream;
  const int pa = prec_a64(precision) ? PV_F64 : PV_F32;
  SVAR_TRY(get_program(h, PROG_A, nrhs, pa, &P, st));
  return run_program(h, *P, const_cast<double*>(v), y, st, nullptr);
}

int svar_apply_P_prec(svar_handle* h, int32_t precision, int32_t nrhs, const double* v, double* z,
                      void* stream) {
  if (!h || !v || !z || nrhs < 1) return inval("bad arguments");
  if (!prec_valid(precision)) return inval("bad precision");
  Program* P = nullptr;
  hipStream_t st = (hipStream_t)stream;
  const int pv = prec_pv_p(precision);
  SVAR_TRY(get_program(h, PROG_P, nrhs, pv, &P, st));
  h->net_off = nullptr;
  return run_program(h, *P, const_cast<double*>(v), z, st, nullptr);
}

int svar_apply_op(svar_handle* h, int32_t op, int32_t nrhs, const double* in, double* out,
                  void* stream) {
  if (!h || !in || !out || nrhs < 1) return inval("bad arguments");
  if (op < SVAR_OP_L || op > SVAR_OP_HT) return inval("unknown operation code");
  if ((op == SVAR_OP_RHAT_INV) && h->popts.type == SVAR_PREC_NONE)
    return inval("Rhat^{-1} needs a preconditioned handle");
  Program* P = nullptr;
  hipStream_t st = (hipStream_t)stream;
  SVAR_TRY(get_program(h, op, nrhs, PV_F64, &P, st));
  return run_program(h, *P, const_cast<double*>(in), out, st, nullptr);
}

int svar_model_forecast(svar_handle* h, int32_t w, const double* x, double* y, void* stream) {
  if (!h || !x || !y || w < 0 || w >= (int)h->wins.size()) return inval("bad arguments");
  if (x == y) return inval("x and y must be distinct");
  hipStream_t st = (hipStream_t)stream;
  const WinDev& W = h->wins[w];
  const ModelDev& M = h->models[W.model_id];
  if (M.kind == MK_L96) {
    launch_l96_forecast(x, y, W.s, W.N, M.F, M.dt, M.nsteps, st);
  } else {
    // linear models: y_i = M_i x_{i-1} through the model-step kernels (y_0 = x_0)
    std::vector<MJob> jobs;
    for (int i = 0; i <= W.N; ++i) {
      MJob J{};
      J.s = W.s;
      J.out = Operand{B_OUT, 0, (int64_t)i * W.s};
      if (i == 0) {
        J.in = Operand{B_IN, 0, 0};
        J.x = J.in;
        J.model = -1;
      } else {
        J.in = Operand{B_AUX, 0, 0};  // zeros
        J.x = Operand{B_IN, 0, (int64_t)(i - 1) * W.s};
        J.model = W.model_id;
        J.mi = i;
        J.alpha = 1.0;
      }
      jobs.push_back(J);
    }
    SVAR_TRY(ensure_zeros(h, W.s, st));
    std::vector<void*> tmp;
    MJob* dj = nullptr;
    SVAR_TRY(upload(tmp, &dj, jobs.data(), jobs.size(), st));
    Bases b{};
    b.p[B_IN] = const_cast<double*>(x);
    b.p[B_OUT] = y;
    b.p[B_AUX] = h->zeros;
    if (M.kind == MK_BAND)
      launch_mstep_band(dj, (int)jobs.size(), W.s, h->max_halo, h->models_dev, b, nullptr, st,
                        h->band_window);
    else
      launch_mstep_dense(dj, (int)jobs.size(), W.s, h->models_dev, b, nullptr, st);
    SVAR_HIP(hipStreamSynchronize(st));
    free_all(tmp);
  }
  SVAR_HIP(hipGetLastError());
  return SVAR_OK;
}

int svar_set_trajectory(svar_handle* h, int32_t w, const double* traj, void* stream) {
  if (!h || !traj || w < 0 || w >= (int)h->wins.size()) return inval("bad arguments");
  const WinDev& W = h->wins[w];
  const ModelDev& M = h->models[W.model_id];
  if (M.kind != MK_L96) return inval("only Lorenz-96 windows carry a trajectory");
  SVAR_HIP(hipMemcpyAsync(const_cast<double*>(M.traj), traj,
                          (size_t)(W.N + 1) * W.s * sizeof(double), hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
  return SVAR_OK;
}

int svar_gn_rhs(svar_handle* h, int32_t w, const double* x, const double* xb, const double* y,
                double* rhs, void* stream) {
  if (!h || !x || !xb || !y || !rhs || w < 0 || w >= (int)h->wins.size())
    return inval("bad arguments");
  hipStream_t st = (hipStream_t)stream;
  const WinDev& W = h->wins[w];
  const int64_t ns = (int64_t)W.nb * W.s;
  double* b = rhs;
  double* d = rhs + ns;
  double* z = rhs + ns + W.P;
  // b_i = M_i(x_{i-1}) - x_i (i >= 1) and b_0 = x_b - x_0
  SVAR_TRY(svar_model_forecast(h, w, x, b, stream));
  launch_axpby(b, x, ns, -1.0, 1.0, st);
  launch_axpby(b, xb, W.s, 1.0, 0.0, st);
  launch_axpby(b, x, W.s, -1.0, 1.0, st);
  // d_i = y_i - H_i x_i
  std::vector<HJob> jobs;
  for (int i = 0; i < W.nb; ++i) {
    if (W.p[i] == 0) continue;
    HJob J{};
    J.x = Operand{B_IN, 0, (int64_t)i * W.s};
    J.out = Operand{B_OUT, 0, (int64_t)W.poff[i]};
    J.cols = W.h_cols + W.h_off[i];
    J.vals = W.h_vals + W.h_off[i];
    J.rows = W.p[i];
    J.width = W.hw;
    jobs.push_back(J);
  }
  if (!jobs.empty()) {
    int mr = 0;
    for (const HJob& J : jobs) mr = std::max(mr, J.rows);
    std::vector<void*> tmp;
    HJob* dj = nullptr;
    SVAR_TRY(upload(tmp, &dj, jobs.data(), jobs.size(), st));
    Bases bb{};
    bb.p[B_IN] = const_cast<double*>(x);
    bb.p[B_OUT] = d;
    launch_gather(dj, (int)jobs.size(), mr, bb, nullptr, st);
    launch_axpby(d, y, W.P, 1.0, -1.0, st);
    SVAR_HIP(hipStreamSynchronize(st));
    free_all(tmp);
  }
  launch_fill(z, ns, 0.0, st);
  SVAR_HIP(hipGetLastError());
  return SVAR_OK;
}

int svar_gn_update(svar_handle* h, int32_t w, double* x, const double* sol, void* stream) {
  if (!h || !x || !sol || w < 0 || w >= (int)h->wins.size()) return inval("bad arguments");
  hipStream_t st = (hipStream_t)stream;
  const WinDev& W = h->wins[w];
  const int64_t ns = (int64_t)W.nb * W.s;
  launch_axpby(x, sol + ns + W.P, ns, 1.0, 1.0, st);
  SVAR_HIP(hipGetLastError());
  if (h->models[W.model_id].kind == MK_L96) return svar_set_trajectory(h, w, x, stream);
  return SVAR_OK;
}

int svar_rhat_params(const svar_handle* h, int32_t w, double* gamma, double* T, double* lam1) {
  if (!h || w < 0 || w >= (int)h->wins.size()) return inval("bad window index");
  const WinDev& W = h->wins[w];
  for (size_t m = 0; m < W.rmats.size(); ++m) {
    const double nan = std::numeric_limits<double>::quiet_NaN();
    if (gamma) gamma[m] = m < W.rr_gamma.size() ? W.rr_gamma[m] : nan;
    if (T) T[m] = m < W.me_T.size() ? W.me_T[m] : nan;
    if (lam1) lam1[m] = m < W.lam1.size() ? W.lam1[m] : nan;
  }
  return SVAR_OK;
}

int svar_timing_enable(svar_handle* h, int32_t kclass, int32_t on) {
  if (!h || kclass < 0 || kclass >= SVAR_KCLASS_COUNT) return inval("bad kernel class");
  h->timers[kclass].on = on != 0;
  return SVAR_OK;
}

int svar_timing_read(svar_handle* h, int32_t kclass, double* total_ms, int64_t* launches,
                     int32_t reset) {
  if (!h || kclass < 0 || kclass >= SVAR_KCLASS_COUNT) return inval("bad kernel class");
  Timer& T = h->timers[kclass];
  for (auto& pr : T.pending) {
    float ms = 0.f;
    SVAR_HIP(hipEventSynchronize(pr.second));
    SVAR_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
    T.total_ms += ms;
    T.pool.push_back(pr);
  }
  T.pending.clear();
  if (total_ms) *total_ms = T.total_ms;
  if (launches) *launches = T.launches;
  if (reset) {
    T.total_ms = 0.0;
    T.launches = 0;
  }
  return SVAR_OK;
}

int svar_destroy(svar_handle* h) {
  if (!h) return SVAR_OK;
  (void)hipDeviceSynchronize();
  for (auto& kv : h->views) svar_destroy(kv.second);  // views own only their programs
  h->views.clear();
  if (h->arena) (void)hipFree(h->arena);
  h->arena = nullptr;
  if (h->graph.exec) (void)hipGraphExecDestroy(h->graph.exec);
  if (h->graph.ev_in) (void)hipEventDestroy(h->graph.ev_in);
  if (h->graph.ev_out) (void)hipEventDestroy(h->graph.ev_out);
  if (h->graph.ps) (void)hipStreamDestroy(h->graph.ps);
  for (auto& T : h->timers) {
    for (auto& pr : T.pending) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    for (auto& pr : T.pool) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  }
  free_all(h->kry.allocs);
  if (h->kry.gl_host) (void)hipHostFree(h->kry.gl_host);
  for (int i = 0; i < 2; ++i)
    if (h->kry.gl_ev[i]) (void)hipEventDestroy(h->kry.gl_ev[i]);
  free_all(h->allocs);
  delete h;
  return SVAR_OK;
}

}  // extern "C"
