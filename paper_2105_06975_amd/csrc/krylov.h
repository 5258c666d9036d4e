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
              hipStream_t st);
void kr_update(const KPlan& p, const KState* stt, const KGlobal* gl, double* V, double* u,
               const double* w, const KHess* hs, int64_t ntot, double* part, int jmax,
               hipStream_t st);
void kr_advance(KGlobal* gl, hipStream_t st);
void kr_solve_y(const KPlan& p, const KState* stt, KHess* hs, int m, hipStream_t st);
void kr_xupdate(const KPlan& p, const KState* stt, const KHess* hs, const double* Zb,
                int64_t ntot, double* x, int m, hipStream_t st);
void kr_resid(double* r, const double* rhs, int64_t n, hipStream_t st);
// workgroups of the Gram-Schmidt passes resident on the current device at once (both passes:
// the smaller of the two), 0 if the runtime cannot tell
int kr_resident_tasks();

}  // namespace svar
