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
// FGMRES over the right-hand sides of a window as one block (k_bkr.hip); P <= KBR_MAX columns
#define KBR_MAX 8
// block steps per cycle: the Hessenberg step and the update keep P^2 (m + 1) doubles in LDS
#define KBR_MAX_CYCLE(P) (7424 / ((P) * (P)) - 1)
#define KBR_TASK 1024   // rows of a window per task of the block passes (256 threads x 4)
struct KBRTask {        // rows [e0, e1) of window `win` (row offsets inside the window)
  int32_t win, pad;
  int64_t off, n;       // packed offset of the window's first column, rows per column
  int64_t e0, e1;
};
struct KBRWin {         // per window, per cycle
  int32_t task0, ntask;
  int32_t done;         // the window's cycle has ended (converged, basis full, breakdown)
  int32_t bad;          // non-finite Gram matrix: breakdown
  int32_t steps;        // block steps taken in this cycle
  int32_t zmask;        // columns of the current block deflated (numerically dependent)
  int32_t rmask;        // deflated columns of the starting block replaced by random vectors
  int32_t cut;          // a new block lost rank: the cycle ends after this step
  int32_t stall, pad;   // learned path: consecutive steps that failed the decrease test
  double prev;          // learned path: the block's residual norm after the previous step
  double Fr[KBR_MAX * KBR_MAX];  // the current Cholesky QR round's factor (row major, upper)
  double Ft[KBR_MAX * KBR_MAX];  // product of the rounds' factors
};
struct KBRHess {        // per window (device pointers), P = the block width
  double* H;            // (m+1) P x m P, column major (column q at q (m+1) P)
  double* cs;           // m P x P rotations: rotation k of column q at q P + k
  double* sn;
  double* G;            // (m+1) P x P right-hand sides of the least-squares problems
  double* Y;            // m P x P solutions
};
struct KBRPlan {
  KBRTask* tasks = nullptr;
  int ntask = 0, nwin = 0;
};
// the block passes (see k_bkr.hip): SLP / SLS are the strides of the per-task partial sums
// and the per-window sums
void bkr_reset(const KBRPlan& p, KBRWin* wins, hipStream_t st);
void bkr_dot(int P, const KBRPlan& p, const KBRWin* wins, const double* A, int64_t lda, int na,
             const double* Wb, double* part, int SLP, hipStream_t st);
void bkr_reduce(const KBRPlan& p, const KBRWin* wins, const double* part, int SLP, int nv,
                double* sums, int SLS, hipStream_t st);
// gpart (nullable): also the per-task Gram partials of the updated block (stride SLP)
void bkr_update(int P, const KBRPlan& p, const KBRWin* wins, const double* A, int64_t lda,
                int na, double* Wb, const double* C, int SLS, double sgn, int final_x,
                double* gpart, int SLP, hipStream_t st);
void bkr_chol(int P, const KBRPlan& p, KBRWin* wins, const double* G, int SLS, int round,
              int start, hipStream_t st);
void bkr_trsm(int P, const KBRPlan& p, const KBRWin* wins, double* Wb, double* gpart, int SLP,
              hipStream_t st);
void bkr_start(int P, const KBRPlan& p, KBRWin* wins, KBRHess* hs, KState* stt,
               const double* tol_rel, const double* G0, int SLS, int m, KGlobal* gl,
               hipStream_t st);
void bkr_hess(int P, const KBRPlan& p, KBRWin* wins, KBRHess* hs, KState* stt, const double* C1,
              const double* C2, int SLS, int j, int m, int* net_off, double drop, int patience,
              HistArg hist, hipStream_t st);
void bkr_solve_y(int P, const KBRPlan& p, const KBRWin* wins, const KBRHess* hs, int m,
                 double* Yl, int SLS, hipStream_t st);
void bkr_flags(int P, const KBRPlan& p, const KBRWin* wins, KGlobal* gl, int* flags,
               int* net_off, hipStream_t st);
// workgroups of the Gram-Schmidt passes resident on the current device at once (both passes:
// the smaller of the two), 0 if the runtime cannot tell
int kr_resident_tasks();

}  // namespace svar
