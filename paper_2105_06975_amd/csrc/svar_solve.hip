// Solve drivers: flexible GMRES cycles inside a float64 refinement loop, and preconditioned
// MINRES (§7: MINRES with P_D, GMRES with P_I, relative two-norm tolerance, x0 = 0).
//
// svar_solve runs cycles of right-preconditioned FGMRES on A d = r with r = rhs - A x
// recomputed in float64 between cycles.  With FP64 operators and no restart this is the
// paper's unrestarted GMRES followed by a true-residual check; with restart it is FGMRES(m);
// with the mixed precisions the inner operators use float32 / bfloat16 covariance products
// while the Arnoldi basis, Hessenberg least squares and residual checks stay float64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>

#include "mem.h"
#include "minres.h"
#include "svar_handle.h"

namespace svar {

// Task plan of the Gram-Schmidt passes.  Every workgroup streams the whole basis over its rows,
// so all tasks run about equally long and a pass proceeds in rounds of `resident` workgroups.
// The fewest tasks of at most KR_TASK rows can leave the last round partly idle (C2 with 8 rhs:
// 2600 tasks on 768 slots fill 3.4 rounds).  The rows are then spread over as many tasks as the
// whole rounds hold, in chunks of 16 rows (128-byte aligned ends), provided every task keeps at
// least 3/4 of KR_TASK rows: a thread loads its KR_EPT elements whatever the task length, so
// short tasks waste loads (measured: 1 rhs of C2, 325 full tasks beat 757 tasks of 880 rows by
// 18 %, while 8 rhs gain 4 % from 3056 tasks of 1744 rows).
static void gs_tasks(const std::vector<int64_t>& ns, int resident, std::vector<KSys>& sys,
                     std::vector<KTask>& tasks) {
  int64_t need = 0;
  for (int64_t n : ns) need += (n + KR_TASK - 1) / KR_TASK;
  double grow = 1.0;
  if (resident > 0 && need > 0) {
    const int64_t rounds = (need + resident - 1) / resident;
    grow = (double)(rounds * resident) / (double)need;
  }
  auto rows_of = [&](int64_t n, double g) {
    const int64_t t0 = (n + KR_TASK - 1) / KR_TASK;
    const int64_t want = std::max<int64_t>(t0, (int64_t)(t0 * g));
    return std::min<int64_t>(KR_TASK, ((n + want - 1) / want + 15) / 16 * 16);
  };
  for (int64_t n : ns)
    if (n >= KR_TASK && 4 * rows_of(n, grow) < 3 * KR_TASK) grow = 1.0;
  sys.assign(ns.size(), KSys{});
  tasks.clear();
  int64_t off = 0;
  for (size_t si = 0; si < ns.size(); ++si) {
    const int64_t n = ns[si];
    const int64_t rows = rows_of(n, grow);
    sys[si].off = off;
    sys[si].n = n;
    sys[si].task0 = (int)tasks.size();
    for (int64_t e = 0; e < n; e += rows) {
      KTask t{};
      t.sys = (int32_t)si;
      t.e0 = off + e;
      t.e1 = off + std::min<int64_t>(n, e + rows);
      tasks.push_back(t);
    }
    sys[si].ntask = (int)tasks.size() - sys[si].task0;
    off += n;
  }
}

// basis stride: ntot rounded to 4 KB plus 12.5 KB, so that consecutive basis vectors do not
// start at the same offset modulo large powers of two (they are read side by side)
static int64_t kry_ldv(int64_t ntot) { return (ntot + 511) / 512 * 512 + 1600; }
// elements of the basis and work vectors of a Krylov workspace of m slots
static int64_t kry_big_elems(int64_t ntot, int m) {
  return 2 * (int64_t)m * kry_ldv(ntot) + 5 * ((ntot + 63) / 64 * 64);
}

int ensure_krylov(svar_handle* h, int nrhs, int m, hipStream_t st) {
  auto& K = h->kry;
  if (K.nrhs == nrhs && K.m >= m) return SVAR_OK;
  SVAR_HIP(hipStreamSynchronize(st));
  // captured step graphs hold the old buffers' addresses: key them on this generation
  ++h->kry_gen;
  free_all(K.allocs);
  {
    KGlobal* keep = K.gl_host;
    hipEvent_t ev0 = K.gl_ev[0], ev1 = K.gl_ev[1];
    K = svar_handle::Kry();
    K.gl_host = keep;
    K.gl_ev[0] = ev0;
    K.gl_ev[1] = ev1;
  }
  const int nw = (int)h->wins.size();
  const int nsys = nw * nrhs;
  const int64_t ntot = handle_total(h, nrhs);
  std::vector<int64_t> ns;
  for (int w = 0; w < nw; ++w)
    for (int r = 0; r < nrhs; ++r) ns.push_back(h->wins[w].n);
  std::vector<KSys> sys;
  std::vector<KTask> tasks;
  gs_tasks(ns, kr_resident_tasks(), sys, tasks);
  K.nrhs = nrhs;
  K.m = m;
  K.ntot = ntot;
  K.ldv = kry_ldv(ntot);
  const int SL = 2 * m + 2;
  auto& A = K.allocs;
  SVAR_TRY(dalloc(A, &K.plan.tasks, tasks.size()));
  SVAR_TRY(dalloc(A, &K.plan.sys, sys.size()));
  SVAR_HIP(hipMemcpyAsync(K.plan.tasks, tasks.data(), tasks.size() * sizeof(KTask),
                          hipMemcpyHostToDevice, st));
  SVAR_HIP(hipMemcpyAsync(K.plan.sys, sys.data(), sys.size() * sizeof(KSys), hipMemcpyHostToDevice,
                          st));
  K.plan.ntask = (int)tasks.size();
  K.plan.nsys = nsys;
  // basis V, Z (m slots of ldv) and the work vectors u, w, z, r, xs in one block: the handle's
  // own allocation, or for a wave's view a carve of the parent's arena
  const int64_t nt64 = (ntot + 63) / 64 * 64;
  double* big = nullptr;
  if (h->parent) {
    if (h->parent->arena_elems < kry_big_elems(ntot, m))
      return inval_msg("wave arena smaller than the wave's Krylov workspace");
    big = h->parent->arena;
  } else {
    SVAR_TRY(dalloc(A, &big, (size_t)kry_big_elems(ntot, m)));
  }
  K.V = big;
  K.Z = K.V + (int64_t)m * K.ldv;
  K.u = K.Z + (int64_t)m * K.ldv;
  K.w = K.u + nt64;
  K.z = K.w + nt64;
  K.r = K.z + nt64;
  K.xs = K.r + nt64;
  SVAR_TRY(dalloc(A, &K.part, (size_t)K.plan.ntask * SL));
  SVAR_TRY(dalloc(A, &K.npart, (size_t)K.plan.ntask));
  SVAR_TRY(dalloc(A, &K.sums, (size_t)nsys * SL));
  SVAR_TRY(dalloc(A, &K.sysv, (size_t)nsys));
  SVAR_TRY(dalloc(A, &K.tol_rel, (size_t)nsys));
  SVAR_TRY(dalloc(A, &K.st, (size_t)nsys));
  SVAR_TRY(dalloc(A, &K.net_off, (size_t)nsys));
  SVAR_TRY(dalloc(A, &K.it0, (size_t)nsys));
  SVAR_TRY(dalloc(A, &K.flags, (size_t)(1 + nsys + nw)));
  SVAR_TRY(dalloc(A, &K.gl, 1));
  // Hessenberg storage per system
  const size_t per = (size_t)(m + 1) * m + m + m + (m + 1) + m + (m + 1) + m;
  SVAR_TRY(dalloc(A, &K.hbuf, per * nsys));
  std::vector<KHess> hs(nsys);
  for (int i = 0; i < nsys; ++i) {
    double* p = K.hbuf + per * i;
    hs[i].H = p;
    p += (size_t)(m + 1) * m;
    hs[i].cs = p;
    p += m;
    hs[i].sn = p;
    p += m;
    hs[i].g = p;
    p += m + 1;
    hs[i].y = p;
    p += m;
    hs[i].hprev = p;
    p += m + 1;
    hs[i].coef_s = p;
  }
  SVAR_TRY(dalloc(A, &K.hs, (size_t)nsys));
  SVAR_HIP(hipMemcpyAsync(K.hs, hs.data(), nsys * sizeof(KHess), hipMemcpyHostToDevice, st));
  if (!K.gl_host) SVAR_HIP(hipHostMalloc((void**)&K.gl_host, 2 * sizeof(KGlobal)));
  for (int i = 0; i < 2; ++i)
    if (!K.gl_ev[i]) SVAR_HIP(hipEventCreateWithFlags(&K.gl_ev[i], hipEventDisableTiming));
  SVAR_HIP(hipStreamSynchronize(st));
  return SVAR_OK;
}

// per-system squared norms of x (host vector)
int sys_norm2(svar_handle* h, const double* x, std::vector<double>& out, hipStream_t st) {
  auto& K = h->kry;
  kr_nrm2_part(K.plan, x, K.npart, st);
  kr_seg_sum(K.plan, K.npart, K.sysv, st);
  out.resize(K.plan.nsys);
  SVAR_HIP(hipMemcpyAsync(out.data(), K.sysv, K.plan.nsys * sizeof(double),
                          hipMemcpyDeviceToHost, st));
  SVAR_HIP(hipStreamSynchronize(st));
  return SVAR_OK;
}

// One FGMRES cycle of at most m iterations on A d = r (K.r), accumulating x += d.
struct Harvest {
  double* buf = nullptr;
  int cap = 0, count = 0;
  int64_t len = 0;
  const Program* prog = nullptr;
};

// One FGMRES step: P and A products, the fused Gram-Schmidt passes and the Hessenberg step.
// The step index itself lives on the device; jl only sizes grids and LDS (any jl >= the
// device's j gives the same results, which lets a captured chunk use jl = m throughout).
static int fg_step(svar_handle* h, int m, const Program& PA, const Program& PP, int jl,
                   bool scale, int* net_off, double drop, int patience, Harvest& hv,
                   HistArg hist, hipStream_t st) {
  auto& K = h->kry;
  const int* skip = &K.gl->all_done;
  if (scale) kr_scale(K.plan, K.npart, K.u, K.st, K.gl, st);
  if (hv.buf && hv.count < hv.cap) {
    SVAR_TRY(run_program(h, *hv.prog, K.u, hv.buf + (int64_t)hv.count * hv.len, st, skip));
    ++hv.count;
  }
  SVAR_TRY(run_program(h, PP, K.u, K.z, st, skip, K.flags));
  SVAR_TRY(run_program(h, PA, K.z, K.w, st, skip, K.flags));
  hipEvent_t e0, e1;
  timed_begin(h, SVAR_KCLASS_ORTHO, st, &e0, &e1);
  kr_dot(K.plan, K.st, K.gl, K.V, K.u, K.w, K.z, K.Z, K.ldv, m, 1, K.part, st);
  timed_end(h, SVAR_KCLASS_ORTHO, st, e0, e1);
  kr_reduce(K.plan, K.st, K.gl, K.part, K.sums, m, jl, st);
  kr_small(K.plan, K.st, K.gl, K.sums, K.hs, m, 0, jl, net_off, drop, patience, hist, st);
  timed_begin(h, SVAR_KCLASS_ORTHO, st, &e0, &e1);
  kr_update(K.plan, K.st, K.gl, K.V, K.u, K.w, K.hs, K.ldv, K.npart, jl, st);
  timed_end(h, SVAR_KCLASS_ORTHO, st, e0, e1);
  kr_advance(K.gl, K.st, K.flags, net_off, K.plan.nsys, K.nrhs, 1, st);
  return SVAR_OK;
}

static constexpr int GRAPH_STEPS = 4;

// The executable graph of GRAPH_STEPS steps for this configuration (captured on first use).
static int step_graph(svar_handle* h, int nrhs, int m, const Program& PA, const Program& PP,
                      int* net_off, double drop, int patience, hipGraphExec_t* out) {
  auto& G = h->graph;
  // every device buffer whose address the captured launches hold
  const void* bufs[6] = {h->kry.V, h->tmp, h->gemm_ws, h->net_ws, h->zeros, h->dz1};
  bool same_bufs = true;
  for (int i = 0; i < 6; ++i) same_bufs = same_bufs && G.bufs[i] == bufs[i];
  if (G.exec && same_bufs && G.nrhs == nrhs && G.m == m && G.pa == &PA && G.pp == &PP &&
      G.gen == h->prog_gen && G.kgen == h->kry_gen && G.net_off == net_off && G.drop == drop &&
      G.patience == patience) {
    *out = G.exec;
    return SVAR_OK;
  }
  if (!G.ps) {
    SVAR_HIP(hipStreamCreateWithFlags(&G.ps, hipStreamNonBlocking));
    SVAR_HIP(hipEventCreateWithFlags(&G.ev_in, hipEventDisableTiming));
    SVAR_HIP(hipEventCreateWithFlags(&G.ev_out, hipEventDisableTiming));
  }
  if (G.exec) {
    SVAR_HIP(hipStreamSynchronize(G.ps));
    (void)hipGraphExecDestroy(G.exec);
    G.exec = nullptr;
  }
  Harvest none;
  hipGraph_t graph = nullptr;
  SVAR_HIP(hipStreamBeginCapture(G.ps, hipStreamCaptureModeThreadLocal));
  int rc = SVAR_OK;
  for (int i = 0; i < GRAPH_STEPS && rc == SVAR_OK; ++i)
    rc = fg_step(h, m, PA, PP, m, true, net_off, drop, patience, none, HistArg(), G.ps);
  hipError_t ce = hipStreamEndCapture(G.ps, &graph);
  if (rc != SVAR_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ce != hipSuccess) {
    set_error(std::string("graph capture failed: ") + hipGetErrorString(ce));
    return SVAR_E_HIP;
  }
  hipError_t ie = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    G.exec = nullptr;
    set_error(std::string("graph instantiation failed: ") + hipGetErrorString(ie));
    return SVAR_E_HIP;
  }
  G.nrhs = nrhs;
  G.m = m;
  G.pa = &PA;
  G.pp = &PP;
  G.gen = h->prog_gen;
  G.kgen = h->kry_gen;
  G.net_off = net_off;
  G.drop = drop;
  G.patience = patience;
  for (int i = 0; i < 6; ++i) G.bufs[i] = bufs[i];
  *out = G.exec;
  return SVAR_OK;
}

// Progress lines on stderr for long solves (environment SVAR_PROGRESS=1): at most one every
// 20 s, from the convergence checks of the FGMRES cycles.
static bool progress_on() {
  static const int on = [] {
    const char* e = std::getenv("SVAR_PROGRESS");
    return e && e[0] == '1' ? 1 : 0;
  }();
  return on != 0;
}
static void progress_line(const svar_handle* h, int j, int remaining) {
  using clk = std::chrono::steady_clock;
  static clk::time_point last = clk::now();
  const clk::time_point now = clk::now();
  if (std::chrono::duration<double>(now - last).count() < 20.0) return;
  last = now;
  const int w0 = h->view_w0;
  std::fprintf(stderr, "svar: windows %d..%d, cycle step %d, %d systems still iterating\n", w0,
               w0 + (int)h->wins.size() - 1, j, remaining);
  std::fflush(stderr);
}

static int fgmres_cycle(svar_handle* h, int nrhs, int m, const Program& PA, const Program& PP,
                        const std::vector<double>& tol_rel, double* x, std::vector<KState>& out,
                        double drop, int patience, Harvest& hv, bool use_graph, HistArg hist,
                        hipStream_t st) {
  int* net_off = h->net_off ? h->kry.net_off : nullptr;
  auto& K = h->kry;
  SVAR_HIP(hipMemcpyAsync(K.tol_rel, tol_rel.data(), tol_rel.size() * sizeof(double),
                          hipMemcpyHostToDevice, st));
  kr_nrm2_part(K.plan, K.r, K.npart, st);
  kr_start(K.plan, K.npart, K.r, K.u, K.st, K.tol_rel, K.gl, st);
  // skip flags of the systems that are inactive in this cycle
  kr_advance(K.gl, K.st, K.flags, net_off, K.plan.nsys, K.nrhs, 0, st);
  const int check_every = GRAPH_STEPS;
  const bool graph = use_graph && !hv.buf && !hist.h && !timing_any(h);
  // Convergence checks: the device flag is copied to the host every check_every steps.  Read
  // at once, the copy drains the queue and the device idles while the host enqueues the next
  // steps; so the host reads each copy one checkpoint later, with the next steps already
  // queued (steps enqueued after every system has converged skip their work).  Harvesting
  // counts its vectors on the host, so it reads each copy at once.
  const bool lagged = !hv.buf;
  bool all_done = false;
  int j = 0, pend = -1, slot = 0;
  while (j < m) {
    int done_steps = 1;
    if (graph && j >= check_every && j % check_every == 0 && j + GRAPH_STEPS <= m) {
      // replay a captured chunk on the private stream, ordered inside the caller's stream
      hipGraphExec_t ex = nullptr;
      SVAR_TRY(step_graph(h, nrhs, m, PA, PP, net_off, drop, patience, &ex));
      SVAR_HIP(hipEventRecord(h->graph.ev_in, st));
      SVAR_HIP(hipStreamWaitEvent(h->graph.ps, h->graph.ev_in, 0));
      SVAR_HIP(hipGraphLaunch(ex, h->graph.ps));
      SVAR_HIP(hipEventRecord(h->graph.ev_out, h->graph.ps));
      SVAR_HIP(hipStreamWaitEvent(st, h->graph.ev_out, 0));
      done_steps = GRAPH_STEPS;
    } else {
      SVAR_TRY(fg_step(h, m, PA, PP, j, j > 0, net_off, drop, patience, hv, hist, st));
    }
    j += done_steps;
    if (j % check_every == 0 || j == m) {
      KGlobal* hb = K.gl_host + slot;
      SVAR_HIP(hipMemcpyAsync(hb, K.gl, sizeof(KGlobal), hipMemcpyDeviceToHost, st));
      SVAR_HIP(hipEventRecord(K.gl_ev[slot], st));
      if (!lagged || j == m) {
        SVAR_HIP(hipEventSynchronize(K.gl_ev[slot]));
        if (hb->all_done || j == m) {
          all_done = hb->all_done != 0;
          break;
        }
        continue;
      }
      if (pend >= 0) {
        SVAR_HIP(hipEventSynchronize(K.gl_ev[pend]));
        if (progress_on()) progress_line(h, j, K.gl_host[pend].remaining);
        if (K.gl_host[pend].all_done) {
          all_done = true;
          break;
        }
      }
      pend = slot;
      slot ^= 1;
    }
  }
  if (!all_done) {
    // every basis slot is used: finalise column m-1 without a new product
    kr_scale(K.plan, K.npart, K.u, K.st, K.gl, st);
    kr_dot(K.plan, K.st, K.gl, K.V, K.u, K.w, K.z, K.Z, K.ldv, m, 0, K.part, st);
    kr_reduce(K.plan, K.st, K.gl, K.part, K.sums, m, m, st);
    kr_small(K.plan, K.st, K.gl, K.sums, K.hs, m, 1, m, net_off, drop, patience, hist, st);
  }
  kr_solve_y(K.plan, K.st, K.hs, m, st);
  kr_xupdate(K.plan, K.st, K.hs, K.Z, K.ldv, x, m, st);
  out.resize(K.plan.nsys);
  SVAR_HIP(hipMemcpyAsync(out.data(), K.st, K.plan.nsys * sizeof(KState), hipMemcpyDeviceToHost,
                          st));
  SVAR_HIP(hipStreamSynchronize(st));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("Krylov kernel failed: ") + hipGetErrorString(e));
    return SVAR_E_HIP;
  }
  return SVAR_OK;
}

static int ensure_block(svar_handle* h) {
  auto& K = h->kry;
  if (K.bpart) return SVAR_OK;
  const int slb = (K.m + 1) * KB_MAX;
  const size_t G = (size_t)KB_MAX * KB_MAX;
  SVAR_TRY(dalloc(K.allocs, &K.bpart, (size_t)K.plan.ntask * slb));
  SVAR_TRY(dalloc(K.allocs, &K.bs1, (size_t)K.plan.nsys * slb));
  SVAR_TRY(dalloc(K.allocs, &K.bs2, (size_t)K.plan.nsys * slb));
  SVAR_TRY(dalloc(K.allocs, &K.gpart, (size_t)K.plan.ntask * G));
  SVAR_TRY(dalloc(K.allocs, &K.gsum, (size_t)K.plan.nsys * G));
  SVAR_TRY(dalloc(K.allocs, &K.kb, (size_t)K.plan.nsys));
  K.slb = slb;
  return SVAR_OK;
}

// One cycle of s-step FGMRES (blocks of s columns, see the block kernels): basis slots
// V[0..m], Z[0..m-1]; the host reads the all-done flag after every block.
static int block_cycle(svar_handle* h, int m, int s, const Program& PA, const Program& PP,
                       const std::vector<double>& tol_rel, double* x, std::vector<KState>& out,
                       double drop, int patience, Harvest& hv, HistArg hist, hipStream_t st) {
  int* net_off = h->net_off ? h->kry.net_off : nullptr;
  SVAR_TRY(ensure_block(h));
  auto& K = h->kry;
  const int B = s <= 4 ? 4 : KB_MAX;
  const int SLB = K.slb;
  const int* skip = &K.gl->all_done;
  SVAR_HIP(hipMemcpyAsync(K.tol_rel, tol_rel.data(), tol_rel.size() * sizeof(double),
                          hipMemcpyHostToDevice, st));
  kr_nrm2_part(K.plan, K.r, K.npart, st);
  kr_start(K.plan, K.npart, K.r, K.V, K.st, K.tol_rel, K.gl, st);
  kr_advance(K.gl, K.st, K.flags, net_off, K.plan.nsys, K.nrhs, 0, st);
  int j = 0;
  while (j < m) {
    const int b = std::min(s, m - j);
    for (int i = 0; i < b; ++i) {
      double* in = K.V + (int64_t)(j + i) * K.ldv;
      double* zo = K.Z + (int64_t)(j + i) * K.ldv;
      double* wo = K.V + (int64_t)(j + i + 1) * K.ldv;
      if (hv.buf && hv.count < hv.cap) {
        SVAR_TRY(run_program(h, *hv.prog, in, hv.buf + (int64_t)hv.count * hv.len, st, skip));
        ++hv.count;
      }
      SVAR_TRY(run_program(h, PP, in, zo, st, skip, K.flags));
      SVAR_TRY(run_program(h, PA, zo, wo, st, skip, K.flags));
      kr_nrm2_part(K.plan, wo, K.npart, st);
      kb_scale(K.plan, K.npart, wo, K.st, K.gl, K.kb, i, st);
    }
    // the ORTHO timing class covers the four passes over the basis (projections, updates)
    double* sums[2] = {K.bs1, K.bs2};
    for (int pass = 0; pass < 2; ++pass) {
      hipEvent_t e0, e1;
      timed_begin(h, SVAR_KCLASS_ORTHO, st, &e0, &e1);
      kb_dot(B, K.plan, K.st, K.gl, K.V, K.ldv, j, b, SLB, K.bpart, st);
      timed_end(h, SVAR_KCLASS_ORTHO, st, e0, e1);
      kb_reduce(K.plan, K.st, K.gl, K.bpart, SLB, (j + 1) * B, sums[pass], st);
      timed_begin(h, SVAR_KCLASS_ORTHO, st, &e0, &e1);
      kb_update(B, K.plan, K.st, K.gl, K.V, K.ldv, j, b, SLB, sums[pass], st);
      timed_end(h, SVAR_KCLASS_ORTHO, st, e0, e1);
    }
    for (int round = 0; round < 2; ++round) {
      kb_gram(B, K.plan, K.st, K.gl, K.V, K.ldv, j, b, K.gpart, st);
      kb_reduce(K.plan, K.st, K.gl, K.gpart, B * B, B * B, K.gsum, st);
      kb_chol(B, K.plan, K.st, K.gl, K.gsum, K.kb, b, round, st);
      kb_trsm(B, K.plan, K.st, K.gl, K.V, K.ldv, j, b, K.kb, st);
    }
    kb_hess(B, K.plan, K.st, K.gl, K.bs1, K.bs2, SLB, K.kb, K.hs, m, j, b, net_off, drop,
            patience, hist, st);
    kr_advance(K.gl, K.st, K.flags, net_off, K.plan.nsys, K.nrhs, 0, st);
    j += b;
    SVAR_HIP(hipMemcpyAsync(K.gl_host, K.gl, sizeof(KGlobal), hipMemcpyDeviceToHost, st));
    SVAR_HIP(hipStreamSynchronize(st));
    if (K.gl_host->all_done) break;
  }
  kr_solve_y(K.plan, K.st, K.hs, m, st);
  kr_xupdate(K.plan, K.st, K.hs, K.Z, K.ldv, x, m, st);
  out.resize(K.plan.nsys);
  SVAR_HIP(hipMemcpyAsync(out.data(), K.st, K.plan.nsys * sizeof(KState), hipMemcpyDeviceToHost,
                          st));
  SVAR_HIP(hipStreamSynchronize(st));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("Krylov kernel failed: ") + hipGetErrorString(e));
    return SVAR_E_HIP;
  }
  return SVAR_OK;
}

// Block FGMRES over the right-hand sides: tasks of KBR_TASK rows per window, per-window states
// and Hessenberg storage for cycles of K.m - 1 block steps.
static int ensure_br(svar_handle* h, hipStream_t st) {
  auto& K = h->kry;
  if (K.br_wins) return SVAR_OK;
  const int P = K.nrhs, m = K.m - 1, nw = (int)h->wins.size();
  std::vector<KBRTask> tasks;
  std::vector<KBRWin> wins(nw);
  int64_t off = 0;
  for (int w = 0; w < nw; ++w) {
    const int64_t n = h->wins[w].n;
    std::memset(&wins[w], 0, sizeof(KBRWin));
    wins[w].task0 = (int)tasks.size();
    for (int64_t e = 0; e < n; e += KBR_TASK) {
      KBRTask t{};
      t.win = w;
      t.off = off;
      t.n = n;
      t.e0 = e;
      t.e1 = std::min<int64_t>(n, e + KBR_TASK);
      tasks.push_back(t);
    }
    wins[w].ntask = (int)tasks.size() - wins[w].task0;
    off += (int64_t)P * n;
  }
  auto& A = K.allocs;
  K.br_slp = std::max(m, 1) * P * P;
  K.br_sls = K.br_slp;
  SVAR_TRY(dalloc(A, &K.br.tasks, tasks.size()));
  SVAR_TRY(dalloc(A, &K.br_wins, (size_t)nw));
  SVAR_HIP(hipMemcpyAsync(K.br.tasks, tasks.data(), tasks.size() * sizeof(KBRTask),
                          hipMemcpyHostToDevice, st));
  SVAR_HIP(hipMemcpyAsync(K.br_wins, wins.data(), nw * sizeof(KBRWin), hipMemcpyHostToDevice, st));
  K.br.ntask = (int)tasks.size();
  K.br.nwin = nw;
  SVAR_TRY(dalloc(A, &K.br_part, (size_t)K.br.ntask * K.br_slp));
  for (double** b : {&K.br_c1, &K.br_c2, &K.br_g0, &K.br_g1, &K.br_yl})
    SVAR_TRY(dalloc(A, b, (size_t)nw * K.br_sls));
  const int64_t ld = (int64_t)(m + 1) * P, mp = (int64_t)m * P;
  const int64_t per = ld * mp + 2 * mp * P + ld * P + mp * P;
  SVAR_TRY(dalloc(A, &K.br_hbuf, (size_t)(per * nw)));
  std::vector<KBRHess> hs(nw);
  for (int w = 0; w < nw; ++w) {
    double* q = K.br_hbuf + per * w;
    hs[w].H = q;
    q += ld * mp;
    hs[w].cs = q;
    q += mp * P;
    hs[w].sn = q;
    q += mp * P;
    hs[w].G = q;
    q += ld * P;
    hs[w].Y = q;
  }
  SVAR_TRY(dalloc(A, &K.br_hs, (size_t)nw));
  SVAR_HIP(hipMemcpyAsync(K.br_hs, hs.data(), nw * sizeof(KBRHess), hipMemcpyHostToDevice, st));
  SVAR_HIP(hipStreamSynchronize(st));
  return SVAR_OK;
}

// One cycle of at most m block steps over the right-hand sides of every window (basis slots
// V[0..m], Z[0..m-1], each holding the whole batch): QR of the residual block, then per step
// Z_j = P^{-1} V_j, W = A Z_j, two block Gram-Schmidt passes, two Cholesky QR rounds and the
// Hessenberg step; the host reads the all-done flag every GRAPH_STEPS steps, one check late.
static int br_cycle(svar_handle* h, int m, int npass, const Program& PA, const Program& PP,
                    const std::vector<double>& tol_rel, double* x, std::vector<KState>& out,
                    double drop, int patience, HistArg hist, hipStream_t st) {
  int* net_off = h->net_off ? h->kry.net_off : nullptr;
  SVAR_TRY(ensure_br(h, st));
  auto& K = h->kry;
  const int P = K.nrhs;
  const KBRPlan& B = K.br;
  const int SLP = K.br_slp, SLS = K.br_sls;
  const int* skip = &K.gl->all_done;
  SVAR_HIP(hipMemcpyAsync(K.tol_rel, tol_rel.data(), tol_rel.size() * sizeof(double),
                          hipMemcpyHostToDevice, st));
  bkr_reset(B, K.br_wins, st);
  double* V0 = K.V;
  SVAR_HIP(hipMemcpyAsync(V0, K.r, K.ntot * sizeof(double), hipMemcpyDeviceToDevice, st));
  double* gram[2] = {K.br_g0, K.br_g1};
  // two Cholesky QR rounds; the Gram partials of round 0 come from the kernel that wrote the
  // block (the last Gram-Schmidt update) unless have_g0 is false, those of round 1 from the
  // first triangular solve
  auto qr = [&](double* Wb, int start, bool have_g0) {
    if (!have_g0) bkr_dot(P, B, K.br_wins, Wb, K.ldv, 1, Wb, K.br_part, SLP, st);
    bkr_reduce(B, K.br_wins, K.br_part, SLP, P * P, gram[0], SLS, st);
    bkr_chol(P, B, K.br_wins, gram[0], SLS, 0, start, st);
    bkr_trsm(P, B, K.br_wins, Wb, K.br_part, SLP, st);
    bkr_reduce(B, K.br_wins, K.br_part, SLP, P * P, gram[1], SLS, st);
    bkr_chol(P, B, K.br_wins, gram[1], SLS, 1, start, st);
    bkr_trsm(P, B, K.br_wins, Wb, nullptr, 0, st);
  };
  qr(V0, 1, false);
  bkr_start(P, B, K.br_wins, K.br_hs, K.st, K.tol_rel, K.br_g0, SLS, m, K.gl, st);
  bkr_flags(P, B, K.br_wins, K.gl, K.flags, net_off, st);
  int pend = -1, slot = 0;
  for (int j = 0; j < m; ++j) {
    double* Vj = K.V + (int64_t)j * K.ldv;
    double* Zj = K.Z + (int64_t)j * K.ldv;
    double* Wn = K.V + (int64_t)(j + 1) * K.ldv;
    SVAR_TRY(run_program(h, PP, Vj, Zj, st, skip, K.flags));
    SVAR_TRY(run_program(h, PA, Zj, Wn, st, skip, K.flags));
    double* C[2] = {K.br_c1, K.br_c2};
    for (int pass = 0; pass < npass; ++pass) {
      hipEvent_t e0, e1;
      timed_begin(h, SVAR_KCLASS_ORTHO, st, &e0, &e1);
      bkr_dot(P, B, K.br_wins, K.V, K.ldv, j + 1, Wn, K.br_part, SLP, st);
      timed_end(h, SVAR_KCLASS_ORTHO, st, e0, e1);
      bkr_reduce(B, K.br_wins, K.br_part, SLP, (j + 1) * P * P, C[pass], SLS, st);
      timed_begin(h, SVAR_KCLASS_ORTHO, st, &e0, &e1);
      bkr_update(P, B, K.br_wins, K.V, K.ldv, j + 1, Wn, C[pass], SLS, -1.0, 0,
                 pass + 1 == npass ? K.br_part : nullptr, SLP, st);
      timed_end(h, SVAR_KCLASS_ORTHO, st, e0, e1);
    }
    qr(Wn, 0, true);
    bkr_hess(P, B, K.br_wins, K.br_hs, K.st, K.br_c1, npass > 1 ? K.br_c2 : nullptr, SLS, j, m,
             net_off, drop,
             patience, hist, st);
    bkr_flags(P, B, K.br_wins, K.gl, K.flags, net_off, st);
    if ((j + 1) % GRAPH_STEPS == 0 && j + 1 < m) {
      KGlobal* hb = K.gl_host + slot;
      SVAR_HIP(hipMemcpyAsync(hb, K.gl, sizeof(KGlobal), hipMemcpyDeviceToHost, st));
      SVAR_HIP(hipEventRecord(K.gl_ev[slot], st));
      if (pend >= 0) {
        SVAR_HIP(hipEventSynchronize(K.gl_ev[pend]));
        if (progress_on()) progress_line(h, j + 1, K.gl_host[pend].remaining * P);
        if (K.gl_host[pend].all_done) break;
      }
      pend = slot;
      slot ^= 1;
    }
  }
  bkr_solve_y(P, B, K.br_wins, K.br_hs, m, K.br_yl, SLS, st);
  bkr_update(P, B, K.br_wins, K.Z, K.ldv, m, x, K.br_yl, SLS, 1.0, 1, nullptr, 0, st);
  out.resize(K.plan.nsys);
  SVAR_HIP(hipMemcpyAsync(out.data(), K.st, K.plan.nsys * sizeof(KState), hipMemcpyDeviceToHost,
                          st));
  SVAR_HIP(hipStreamSynchronize(st));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("Krylov kernel failed: ") + hipGetErrorString(e));
    return SVAR_E_HIP;
  }
  return SVAR_OK;
}

static int solve_fgmres(svar_handle* h, const svar_solve_opts* o, int nrhs, const double* rhs,
                        double* x, svar_solve_info* info, hipStream_t st) {
  const int nsys = (int)h->wins.size() * nrhs;
  // one cycle holds at most KR_MAX_CYCLE basis vectors (LDS of the update pass); longer
  // unrestarted runs continue as further cycles of the refinement loop
  // block mode (s-step) when block >= 2; its cycles hold at most KB_MAX_CYCLE
  // columns (LDS of the Hessenberg step) and use basis slots 0..m
  const int blk = o->block >= 2 ? std::min((int)o->block, KB_MAX) : 0;
  const bool brhs = o->block_rhs != 0;
  const int cap = brhs ? KBR_MAX_CYCLE(nrhs) : (blk ? KB_MAX_CYCLE : KR_MAX_CYCLE);
  int cyc = o->restart > 0 ? std::min(o->restart, o->maxit) : o->maxit;
  cyc = std::min(cyc, cap);
  if (cyc < 1) return inval_msg("maxit must be >= 1");
  // the workspace holds a full restart cycle even when maxit is smaller, so that a short first
  // call builds what later calls with the same restart use
  const int ws_m = o->restart > 0 ? std::min((int)o->restart, cap) : cyc;
  SVAR_TRY(ensure_krylov(h, nrhs, (blk || brhs) ? ws_m + 1 : ws_m, st));
  auto& K = h->kry;
  // inner operators: FP64_F32P / FP64_BF16P keep A in float64 (no refinement needed: under flexible GMRES
  // the preconditioner's rounding changes only the convergence rate, not the attainable
  // residual); the MIXED settings use float32 A and refine in float64
  const bool a64 = prec_a64(o->precision);
  const int pv_a = a64 ? PV_F64 : PV_F32;
  const int pv_p = prec_pv_p(o->precision);
  Program *A64 = nullptr, *Ain = nullptr, *Pin = nullptr;
  SVAR_TRY(get_program(h, PROG_A, nrhs, PV_F64, &A64, st));
  if (h->popts.type == SVAR_PREC_PI && (a64 || o->precision == SVAR_PRECISION_MIXED_F32)) {
    // every inner A z follows z = P_I u at once: P keeps D z1 (float64, or float32 for
    // MIXED_F32) and A reuses it
    SVAR_TRY(get_program(h, PROG_AD, nrhs, a64 ? PV_F64 : PV_F32, &Ain, st));
    SVAR_TRY(get_program(h, PROG_PD, nrhs, a64 ? pv_p : PV_F32ALL, &Pin, st));
  } else {
    SVAR_TRY(get_program(h, PROG_A, nrhs, pv_a, &Ain, st));
    SVAR_TRY(get_program(h, PROG_P, nrhs, pv_p, &Pin, st));
  }
  launch_fill(x, K.ntot, 0.0, st);
  // learned correction: per-system switch-off flags, cleared for this solve
  const double drop = o->fallback_drop;
  h->net_off = nullptr;
  if (h->net) {  // fallback bits (drop > 0) and done bits, see k_fg_advance
    net_fill_int(K.net_off, nsys, 0, st);
    h->net_off = K.net_off;
  }
  Harvest hv;
  if (o->harvest && o->harvest_cap > 0) {
    SVAR_TRY(get_program(h, PROG_HARVEST, nrhs, PV_F64, const_cast<Program**>(&hv.prog), st));
    hv.buf = o->harvest;
    hv.cap = o->harvest_cap;
    hv.len = state_total(h, nrhs);
  }
  HistArg hist;
  if (o->history && o->history_len > 0) {
    hist.h = o->history;
    hist.len = o->history_len;
    hist.it0 = K.it0;
    launch_fill(o->history, (int64_t)nsys * o->history_len,
                std::numeric_limits<double>::quiet_NaN(), st);
  }
  std::vector<double> rhs2;
  SVAR_TRY(sys_norm2(h, rhs, rhs2, st));
  std::vector<int> iters(nsys, 0), status(nsys, SVAR_OK), cycles(nsys, 0), fallbacks(nsys, 0);
  std::vector<double> est(nsys, 0.0), relres(nsys, 1.0);
  for (int i = 0; i < nsys; ++i) {
    relres[i] = rhs2[i] > 0 ? 1.0 : 0.0;
    if (!std::isfinite(rhs2[i])) status[i] = SVAR_E_BREAKDOWN;  // non-finite right-hand side
  }
  SVAR_HIP(hipMemcpyAsync(K.r, rhs, K.ntot * sizeof(double), hipMemcpyDeviceToDevice, st));
  int64_t applies_A64 = 0;
  int max_outer = std::max(1, o->max_outer);
  if (o->restart <= 0 && o->maxit > cap)
    max_outer = std::max(max_outer, (o->maxit + cap - 1) / cap + 1);
  // a block cut short (rank-deficient block) ends its cycle early: restarts then continue
  // until maxit iterations are used
  if (blk) max_outer = std::max(max_outer, o->maxit);
  int used = 0;
  for (int outer = 0; outer < max_outer; ++outer) {
    std::vector<double> r2 = rhs2;
    if (outer > 0) {
      SVAR_TRY(run_program(h, *A64, x, K.r, st, nullptr));
      kr_resid(K.r, rhs, K.ntot, st);
      ++applies_A64;
      SVAR_TRY(sys_norm2(h, K.r, r2, st));
    }
    bool all = true;
    std::vector<double> tol(nsys);
    for (int i = 0; i < nsys; ++i) {
      const double nr = std::sqrt(r2[i]), nb = std::sqrt(rhs2[i]);
      relres[i] = nb > 0 ? nr / nb : 0.0;
      const bool ok = relres[i] <= o->rtol;
      if (!std::isfinite(relres[i])) status[i] = SVAR_E_BREAKDOWN;
      if (ok || status[i] == SVAR_E_BREAKDOWN || iters[i] >= o->maxit) {
        tol[i] = 2.0;  // inactive in this cycle
        continue;
      }
      all = false;
      double t = nr > 0 ? o->rtol * nb / nr : 1.0;
      if (!a64) t = std::max(t, o->inner_rtol);
      tol[i] = t;
    }
    if (all) break;
    const int m = std::min(cyc, o->maxit - used);
    if (m < 1) break;
    std::vector<KState> ks;
    if (hist.h)
      SVAR_HIP(hipMemcpyAsync(K.it0, iters.data(), nsys * sizeof(int), hipMemcpyHostToDevice, st));
    {
      const int rc = brhs  ? br_cycle(h, m, o->block_rhs == 2 ? 1 : 2, *Ain, *Pin, tol, x, ks,
                                      drop, o->fallback_patience, hist, st)
                     : blk ? block_cycle(h, m, blk, *Ain, *Pin, tol, x, ks, drop,
                                         o->fallback_patience, hv, hist, st)
                           : fgmres_cycle(h, nrhs, m, *Ain, *Pin, tol, x, ks, drop,
                                          o->fallback_patience, hv, o->use_graph != 0, hist, st);
      if (rc != SVAR_OK) {
        h->net_off = nullptr;
        return rc;
      }
    }
    int jmax = 0;
    for (int i = 0; i < nsys; ++i) {
      // a block over the right-hand sides carries a window's converged columns along: they
      // take the window's steps (one P and one A product each)
      if (tol[i] >= 1.0 && !(brhs && ks[i].iters > 0)) continue;
      iters[i] += ks[i].iters;
      cycles[i] += 1;
      fallbacks[i] = std::max(fallbacks[i], (int)ks[i].fallback);
      est[i] = ks[i].est / std::max(std::sqrt(rhs2[i]), 1e-300);
      if (ks[i].status == SVAR_E_BREAKDOWN) status[i] = SVAR_E_BREAKDOWN;
      jmax = std::max(jmax, ks[i].iters);
    }
    used += std::max(jmax, 1);
  }
  h->net_off = nullptr;
  // final true residual in float64
  SVAR_TRY(run_program(h, *A64, x, K.r, st, nullptr));
  kr_resid(K.r, rhs, K.ntot, st);
  ++applies_A64;
  std::vector<double> r2;
  SVAR_TRY(sys_norm2(h, K.r, r2, st));
  int rc = SVAR_OK;
  for (int i = 0; i < nsys; ++i) {
    const double nb = std::sqrt(rhs2[i]);
    const double rr = !std::isfinite(nb) ? std::numeric_limits<double>::quiet_NaN()
                                         : (nb > 0 ? std::sqrt(r2[i]) / nb : 0.0);
    svar_solve_info& I = info[i];
    I.iters = iters[i];
    I.outer = cycles[i];
    I.relres_true = rr;
    I.relres_est = est[i];
    I.status = status[i];
    I.fallbacks = fallbacks[i];
    if (I.status == SVAR_OK && !(rr <= o->rtol)) I.status = std::isfinite(rr) ? SVAR_E_NOCONV
                                                                            : SVAR_E_BREAKDOWN;
    const double per_rhs = 1.0 / (double)nsys;
    (void)per_rhs;
    // component products per system, as counted in Tables 4 and 5 (per right-hand side)
    const int nw = (int)h->wins.size();
    const double scale = 1.0 / (double)(nw * nrhs);
    I.n_M = (int64_t)std::llround((Ain->cnt[0] + Pin->cnt[0]) * scale * iters[i] +
                                  A64->cnt[0] * scale * applies_A64);
    I.n_MT = (int64_t)std::llround((Ain->cnt[1] + Pin->cnt[1]) * scale * iters[i] +
                                   A64->cnt[1] * scale * applies_A64);
    I.n_D = (int64_t)std::llround((Ain->cnt[2] + Pin->cnt[2]) * scale * iters[i] +
                                  A64->cnt[2] * scale * applies_A64);
    I.n_R = (int64_t)std::llround((Ain->cnt[3] + Pin->cnt[3]) * scale * iters[i] +
                                  A64->cnt[3] * scale * applies_A64);
    I.n_Rhat_inv = (int64_t)std::llround(Pin->cnt[4] * scale * iters[i]);
    I.n_Dhat_inv = (int64_t)std::llround(Pin->cnt[5] * scale * iters[i]);
    if (I.status != SVAR_OK && rc == SVAR_OK) rc = I.status;
  }
  if (rc != SVAR_OK) set_error("at least one system did not reach rtol (see info)");
  return rc;
}

// ------------------------------------------------------------------ wave scheduling
// A view over windows [w0, w1) of h: shares the matrices, model tables and zero buffer, and
// builds its own launch programs (created on first use, owned by h).
int get_view(svar_handle* h, int w0, int w1, svar_handle** out) {
  auto it = h->views.find({w0, w1});
  if (it != h->views.end()) {
    *out = it->second;
    return SVAR_OK;
  }
  svar_handle* v = new svar_handle();
  v->device = h->device;
  v->popts = h->popts;
  v->wins.assign(h->wins.begin() + w0, h->wins.begin() + w1);
  v->models = h->models;
  v->models_dev = h->models_dev;
  v->max_halo = h->max_halo;
  v->l96_max_steps = h->l96_max_steps;
  v->band_window = h->band_window;
  v->zeros = h->zeros;
  v->zeros_elems = h->zeros_elems;
  v->net = h->net;
  v->tune = h->tune;
  v->parent = h;
  v->view_w0 = w0;
  h->views[{w0, w1}] = v;
  *out = v;
  return SVAR_OK;
}

// Contiguous waves of windows whose packed length stays within the limit (opts.wave_len, or
// what the free device memory holds at (2 m + 8) doubles per element: the basis, work vectors
// and the views' own buffers).  One wave when everything fits.
static int plan_waves(svar_handle* h, const svar_solve_opts* o, int nrhs, int m,
                      std::vector<std::pair<int, int>>& waves) {
  const int nw = (int)h->wins.size();
  int64_t limit = o->wave_len;
  if (limit <= 0) {
    size_t fr = 0, tot = 0;
    SVAR_HIP(hipMemGetInfo(&fr, &tot));
    // memory this handle already holds for Krylov vectors is available to the solve
    int64_t held = h->arena_elems;
    if (h->kry.nrhs > 0) held += kry_big_elems(h->kry.ntot, h->kry.m);
    const double avail = 0.85 * ((double)fr + 8.0 * (double)held);
    limit = (int64_t)(avail / (8.0 * (2.0 * m + 8.0)));
  }
  waves.clear();
  int w0 = 0;
  int64_t acc = 0;
  for (int w = 0; w < nw; ++w) {
    const int64_t len = (int64_t)nrhs * h->wins[w].n;
    if (w > w0 && acc + len > limit) {
      waves.push_back({w0, w});
      w0 = w;
      acc = 0;
    }
    acc += len;
  }
  waves.push_back({w0, nw});
  return SVAR_OK;
}

// Views that the current wave plan does not use are destroyed (their launch programs and Krylov
// buffers); with a single wave the arena goes too, since the handle then solves in its own
// workspace and the plan counted the arena as free memory.
static int drop_views(svar_handle* h, const std::vector<std::pair<int, int>>& waves,
                      hipStream_t st) {
  const bool single = waves.size() <= 1;
  bool sync = false;
  for (auto it = h->views.begin(); it != h->views.end();) {
    const bool used = !single && std::find(waves.begin(), waves.end(), it->first) != waves.end();
    if (used) {
      ++it;
      continue;
    }
    if (!sync) {
      SVAR_HIP(hipStreamSynchronize(st));
      sync = true;
    }
    svar_destroy(it->second);
    it = h->views.erase(it);
  }
  if (single && h->arena) {
    if (!sync) SVAR_HIP(hipStreamSynchronize(st));
    (void)hipFree(h->arena);
    h->arena = nullptr;
    h->arena_elems = 0;
  }
  return SVAR_OK;
}

static int solve_waves(svar_handle* h, const svar_solve_opts* o, int nrhs, const double* rhs,
                       double* x, svar_solve_info* info, hipStream_t st, int m,
                       const std::vector<std::pair<int, int>>& waves) {
  if (o->harvest && o->harvest_cap > 0)
    return inval_msg("harvesting needs one wave (raise wave_len)");
  std::vector<int64_t> off(h->wins.size() + 1);
  SVAR_TRY(svar_offsets(h, nrhs, off.data()));
  // the arena holds the largest wave's basis and work vectors
  int64_t need = 0;
  for (const auto& wv : waves) need = std::max(need, kry_big_elems(off[wv.second] - off[wv.first], m));
  if (h->kry.nrhs > 0) {  // the handle's own single-wave workspace is not needed in waves
    SVAR_HIP(hipStreamSynchronize(st));
    free_all(h->kry.allocs);
    h->kry.nrhs = -1;
    ++h->kry_gen;
  }
  if (need > h->arena_elems) {
    SVAR_HIP(hipStreamSynchronize(st));
    for (auto& kv : h->views) {  // their carves point into the old arena
      free_all(kv.second->kry.allocs);
      kv.second->kry.nrhs = -1;
      ++kv.second->kry_gen;
    }
    if (h->arena) (void)hipFree(h->arena);
    h->arena = nullptr;
    h->arena_elems = 0;
    if (hipMalloc((void**)&h->arena, (size_t)need * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      h->arena = nullptr;
      set_error("device allocation of the wave arena failed (" + std::to_string(need) +
                " doubles)");
      return SVAR_E_NOMEM;
    }
    h->arena_elems = need;
  }
  int rc = SVAR_OK;
  std::string first_err;
  for (const auto& wv : waves) {
    svar_handle* v = nullptr;
    SVAR_TRY(get_view(h, wv.first, wv.second, &v));
    if (v->net != h->net) SVAR_TRY(svar_set_net(v, h->net));
    svar_solve_opts ow = *o;
    ow.wave_len = 0;
    if (o->history && o->history_len > 0)
      ow.history = o->history + (int64_t)wv.first * nrhs * o->history_len;
    const int64_t b = off[wv.first];
    const int r = solve_fgmres(v, &ow, nrhs, rhs + b, x + b, info + (int64_t)wv.first * nrhs, st);
    if (r != SVAR_OK && r != SVAR_E_NOCONV && r != SVAR_E_BREAKDOWN) return r;
    if (r != SVAR_OK && rc == SVAR_OK) {
      rc = r;
      first_err = svar_last_error();
    }
  }
  if (rc != SVAR_OK) set_error(first_err);
  return rc;
}

}  // namespace svar

using namespace svar;

extern "C" int svar_solve(svar_handle* h, const svar_solve_opts* o, int32_t nrhs,
                          const double* rhs, double* x, svar_solve_info* info, void* stream) {
  if (!h || !o || !rhs || !x || !info || nrhs < 1) return inval_msg("bad arguments");
  if (!(o->rtol > 0.0) || o->maxit < 1) return inval_msg("need rtol > 0 and maxit >= 1");
  if (!prec_valid(o->precision)) return inval_msg("bad precision");
  hipStream_t st = (hipStream_t)stream;
  if (o->wave_len < 0) return inval_msg("wave_len must be >= 0");
  if (o->block_rhs != 0) {
    if (o->block_rhs < 0 || o->block_rhs > 2) return inval_msg("block_rhs must be 0, 1 or 2");
    if (o->method != SVAR_METHOD_FGMRES) return inval_msg("block_rhs needs FGMRES");
    if (nrhs > KBR_MAX) return inval_msg("block_rhs takes at most 8 right-hand sides");
    if (o->block >= 2) return inval_msg("block_rhs and block (s-step) exclude each other");
    if (o->harvest && o->harvest_cap > 0) return inval_msg("block_rhs does not harvest");
  }
  if (o->method == SVAR_METHOD_FGMRES) {
    // basis slots of one cycle, as in solve_fgmres
    const int blk = o->block >= 2 ? std::min((int)o->block, KB_MAX) : 0;
    const bool brhs = o->block_rhs != 0;
    const int cap = brhs ? KBR_MAX_CYCLE(nrhs) : (blk ? KB_MAX_CYCLE : KR_MAX_CYCLE);
    int cyc = o->restart > 0 ? std::min(o->restart, cap) : std::min(o->maxit, cap);
    const int slots = (blk || brhs) ? cyc + 1 : cyc;
    std::vector<std::pair<int, int>> waves;
    if (h->wins.size() > 1) SVAR_TRY(plan_waves(h, o, nrhs, slots, waves));
    SVAR_TRY(drop_views(h, waves, st));
    if (waves.size() > 1) return solve_waves(h, o, nrhs, rhs, x, info, st, slots, waves);
    return solve_fgmres(h, o, nrhs, rhs, x, info, st);
  }
  if (o->method == SVAR_METHOD_MINRES) {
    if (h->popts.type == SVAR_PREC_PI)
      return inval_msg("MINRES needs a symmetric positive definite preconditioner (P_D)");
    if (o->precision != SVAR_PRECISION_FP64) return inval_msg("MINRES runs in float64 only");
    return solve_minres(h, o, nrhs, rhs, x, info, st);
  }
  return inval_msg("bad method");
}
