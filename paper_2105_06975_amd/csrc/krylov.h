// Internal declarations of the device Krylov solvers.
#pragma once
#include "svar_impl.h"

namespace svar {

#define KR_EPT 8                 // elements per thread of the Gram-Schmidt passes
#define KR_TASK (256 * KR_EPT)   // elements per task (workgroup) of a pass
#define KR_MAX_CYCLE 2500        // basis vectors per FGMRES cycle (LDS of the small steps)

struct KTask {      // a contiguous element range of one system
  int32_t sys, pad;
  int64_t e0, e1;   // absolute offsets in the packed vector
};
struct KSys {
  int64_t off, n;
  int32_t task0, ntask;
};
struct KState {     // per system, per cycle
  int32_t done, iters, status, fallback;  // fallback: the learned correction was switched off
  double beta;      // norm of the cycle's initial residual
  double tol_abs;   // stop when the residual estimate is <= tol_abs
  double sigma;     // scale applied to the current candidate u_j
  double nu;        // norm of the re-orthogonalised candidate
  double est;       // latest residual estimate
  int32_t stall;    // consecutive steps that failed the learned path's decrease test
  int32_t pad2;
};
struct KGlobal {
  int32_t j, remaining, all_done, pad;
};
struct KHess {      // per-system dense storage (device pointers)
  double* H;        // (m+1) x m, column major (column c at c*(m+1))
  double* cs;
  double* sn;
  double* g;        // m+1
  double* y;        // m
  double* hprev;    // m+1: provisional column
  double* coef_s;   // m: re-orthogonalisation coefficients
};
// s-step (block) FGMRES: per-system state of the current block of at most KB_MAX columns
#define KB_MAX 8
#define KB_MAX_CYCLE 768   // columns per cycle in block mode (LDS of the Hessenberg step)
struct KBlock {
  double d[KB_MAX];             // norms of the block's products A z before normalisation
  double Rc[KB_MAX * KB_MAX];   // the current Cholesky QR round's factor (row major, upper)
  double R[KB_MAX * KB_MAX];    // product of the rounds' factors
  int32_t blen, pad;            // leading columns that passed both Cholesky rounds
};
// residual history of a solve (see svar_solve_opts.history): h[sys * len + it0[sys] + t]
// receives the residual estimate after step t of the current cycle; h == nullptr: off
struct HistArg {
  double* h = nullptr;
  int len = 0, pad = 0;
  const int* it0 = nullptr;  // device, per system: iterations done in earlier cycles
};
struct KPlan {
  KTask* tasks = nullptr;
  KSys* sys = nullptr;
  int ntask = 0, nsys = 0;
};

void kr_nrm2_part(const KPlan& p, const double* x, double* part, hipStream_t st);
void kr_seg_sum(const KPlan& p, const double* part, double* out, hipStream_t st);
void kr_start(const KPlan& p, const double* part, const double* r, double* u, KState* stt,
              const double* tol_rel, KGlobal* gl, hipStream_t st);
void kr_scale(const KPlan& p, const double* part, double* u, KState* stt, KGlobal* gl,
              hipStream_t st);
void kr_dot(const KPlan& p, const KState* stt, const KGlobal* gl, const double* V,
            const double* u, const double* w, const double* z, double* Zb, int64_t ntot, int m,
            int with_w, double* part, hipStream_t st);
void kr_reduce(const KPlan& p, const KState* stt, const KGlobal* gl, const double* part,
               double* sums, int m, int jmax, hipStream_t st);
void kr_small(const KPlan& p, KState* stt, KGlobal* gl, const double* sums, KHess* hs, int m,
              int finalize_only, int jmax, int* net_off, double drop, int patience,
              HistArg hist, hipStream_t st);
void kr_update(const KPlan& p, const KState* stt, const KGlobal* gl, double* V, double* u,
               const double* w, const KHess* hs, int64_t ntot, double* part, int jmax,
               hipStream_t st);
// advance j (advance != 0) and refresh the operator skip flags and the done bit of the
// network switch-off flags (both nullable, see k_fg_advance)
void kr_advance(KGlobal* gl, const KState* stt, int* flags, int* net_off, int nsys, int nrhs,
                int advance, hipStream_t st);
void kr_solve_y(const KPlan& p, const KState* stt, KHess* hs, int m, hipStream_t st);
void kr_xupdate(const KPlan& p, const KState* stt, const KHess* hs, const double* Zb,
                int64_t ntot, double* x, int m, hipStream_t st);
void kr_resid(double* r, const double* rhs, int64_t n, hipStream_t st);
// block mode (s-step FGMRES); B = KB_MAX or 4 (template width), b <= B columns, basis slots:
// V[0..j] orthonormal, V[j+1..j+b] the block W, Z[j..j+b-1] its preconditioned inputs
void kb_scale(const KPlan& p, const double* part, double* x, const KState* stt,
              const KGlobal* gl, KBlock* kb, int i, hipStream_t st);
void kb_dot(int B, const KPlan& p, const KState* stt, const KGlobal* gl, const double* V,
            int64_t ldv, int j, int b, int SLB, double* part, hipStream_t st);
void kb_reduce(const KPlan& p, const KState* stt, const KGlobal* gl, const double* part, int SL,
               int nused, double* sums, hipStream_t st);
void kb_update(int B, const KPlan& p, const KState* stt, const KGlobal* gl, double* V,
               int64_t ldv, int j, int b, int SLB, const double* C, hipStream_t st);
void kb_gram(int B, const KPlan& p, const KState* stt, const KGlobal* gl, const double* V,
             int64_t ldv, int j, int b, double* part, hipStream_t st);
void kb_chol(int B, const KPlan& p, const KState* stt, const KGlobal* gl, const double* gsum,
             KBlock* kb, int b, int round, hipStream_t st);
void kb_trsm(int B, const KPlan& p, const KState* stt, const KGlobal* gl, double* V, int64_t ldv,
             int j, int b, const KBlock* kb, hipStream_t st);
void kb_hess(int B, const KPlan& p, KState* stt, KGlobal* gl, const double* S1, const double* S2,
             int SLB, const KBlock* kb, KHess* hs, int m, int j, int b, int* net_off,
             double drop, int patience, HistArg hist, hipStream_t st);
// workgroups of the Gram-Schmidt passes resident on the current device at once (both passes:
// the smaller of the two), 0 if the runtime cannot tell
int kr_resident_tasks();

}  // namespace svar
