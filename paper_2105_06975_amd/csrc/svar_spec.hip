// Spectral diagnostics: Lanczos estimates of the eigenvalues of the preconditioned blocks that
// the paper's bounds are stated for (Theorem 1: P_D^{-1} A; Propositions 3-4: Rhat^{-1} R;
// Propositions 1-2: L_M(k)^{-T} L^T L L_M(k)^{-1}).
//
// For K symmetric and M symmetric positive definite with M^{-1} available, the Lanczos process in
// the M inner product (the recurrence of preconditioned MINRES) builds a tridiagonal T_j whose
// eigenvalues (Ritz values) approximate those of M^{-1} K, the extreme ones first:
//   r_1 = start, z_1 = M^{-1} r_1, beta_1 = sqrt(r_1^T z_1);
//   step j: v_j = z_j / beta_j, p = K v_j, alpha_j = v_j^T p,
//           p -= alpha_j r_j / beta_j + beta_j r_{j-1} / beta_{j-1},
//           z_{j+1} = M^{-1} p, beta_{j+1} = sqrt(p^T z_{j+1}), r_{j+1} = p.
// No re-orthogonalisation: lost orthogonality shows as repeated copies of converged Ritz values,
// which leaves the extreme ones intact.  T_j's eigenvalues are found by bisection on Sturm
// sequence counts.
#include <algorithm>
#include <cmath>
#include <vector>

#include "mem.h"
#include "setup.h"
#include "svar_handle.h"

namespace svar {
namespace {

// number of eigenvalues of the symmetric tridiagonal (a, b) below x (Sturm sequence)
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
    q = a[i] - x - (i > 0 ? bb / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

std::vector<double> tridiag_eigs(const std::vector<double>& a, const std::vector<double>& b) {
  const int n = (int)a.size();
  double lo = 0.0, hi = 0.0;
  for (int i = 0; i < n; ++i) {  // Gershgorin interval
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = i == 0 ? a[i] - r : std::min(lo, a[i] - r);
    hi = i == 0 ? a[i] + r : std::max(hi, a[i] + r);
  }
  const double pad = 1e-12 * std::max(std::fabs(lo), std::fabs(hi)) + 1e-300;
  lo -= pad;
  hi += pad;
  std::vector<double> ev(n);
  for (int k = 0; k < n; ++k) {  // the (k+1)-th smallest: count(x) > k
    double l = lo, u = hi;
    for (int it = 0; it < 200 && u - l > 1e-15 * std::max(std::fabs(l), std::fabs(u)); ++it) {
      const double m = 0.5 * (l + u);
      if (sturm_count(a, b, m) > k)
        u = m;
      else
        l = m;
    }
    ev[k] = 0.5 * (l + u);
  }
  return ev;
}

int dot(const double* x, const double* y, int64_t n, double* part, hipStream_t st, double* out) {
  const int g = su_dot_part(x, y, n, part, st);
  std::vector<double> hp(g);
  SVAR_HIP(hipMemcpyAsync(hp.data(), part, g * sizeof(double), hipMemcpyDeviceToHost, st));
  SVAR_HIP(hipStreamSynchronize(st));
  double s = 0.0;
  for (double v : hp) s += v;
  *out = s;
  return SVAR_OK;
}

}  // namespace
}  // namespace svar

using namespace svar;

extern "C" int svar_spectrum(svar_handle* h, int32_t which, int32_t w, int32_t nsteps,
                             const double* start, double* ritz, int32_t* nritz, void* stream) {
  if (!h || !start || !ritz || !nritz || nsteps < 1) return inval_msg("bad arguments");
  if (w < 0 || w >= (int)h->wins.size()) return inval_msg("bad window index");
  if (which == SVAR_SPEC_PD_A && h->popts.type != SVAR_PREC_PD)
    return inval_msg("P_D^{-1} A needs a P_D handle");
  if (which == SVAR_SPEC_RHAT_R && h->popts.type == SVAR_PREC_NONE)
    return inval_msg("Rhat^{-1} R needs a preconditioned handle");
  if (which < SVAR_SPEC_PD_A || which > SVAR_SPEC_LML) return inval_msg("bad spectrum kind");
  hipStream_t st = (hipStream_t)stream;
  svar_handle* v = h;
  if (h->wins.size() > 1) SVAR_TRY(get_view(h, w, w + 1, &v));
  const WinDev& W = v->wins[0];
  const int64_t n = which == SVAR_SPEC_PD_A ? W.n
                    : which == SVAR_SPEC_RHAT_R ? (int64_t)W.P
                                                : (int64_t)W.nb * W.s;
  if (n < 1) return inval_msg("empty operator space");
  // programs: K and M^{-1}
  Program *K1 = nullptr, *K2 = nullptr, *K3 = nullptr, *K4 = nullptr, *Mi = nullptr;
  if (which == SVAR_SPEC_PD_A) {
    SVAR_TRY(get_program(v, PROG_A, 1, PV_F64, &K1, st));
    SVAR_TRY(get_program(v, PROG_P, 1, PV_F64, &Mi, st));
  } else if (which == SVAR_SPEC_RHAT_R) {
    SVAR_TRY(get_program(v, SVAR_OP_R, 1, PV_F64, &K1, st));
    SVAR_TRY(get_program(v, SVAR_OP_RHAT_INV, 1, PV_F64, &Mi, st));
  } else {
    SVAR_TRY(get_program(v, SVAR_OP_LHAT_INV, 1, PV_F64, &K1, st));
    SVAR_TRY(get_program(v, SVAR_OP_L, 1, PV_F64, &K2, st));
    SVAR_TRY(get_program(v, SVAR_OP_LT, 1, PV_F64, &K3, st));
    SVAR_TRY(get_program(v, SVAR_OP_LHAT_INVT, 1, PV_F64, &K4, st));
  }
  std::vector<void*> tmp;
  double *r_prev = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *t1 = nullptr,
         *t2 = nullptr, *part = nullptr;
  int rc = SVAR_OK;
  for (double** b : {&r_prev, &r, &z, &p, &t1, &t2})
    if (rc == SVAR_OK) rc = dalloc(tmp, b, (size_t)n);
  if (rc == SVAR_OK) rc = dalloc(tmp, &part, (size_t)2048);
  auto applyK = [&](double* x, double* y) -> int {
    if (which != SVAR_SPEC_LML) return run_program(v, *K1, x, y, st, nullptr);
    SVAR_TRY(run_program(v, *K1, x, t1, st, nullptr));   // L_M^{-1} x
    SVAR_TRY(run_program(v, *K2, t1, t2, st, nullptr));  // L L_M^{-1} x
    SVAR_TRY(run_program(v, *K3, t2, t1, st, nullptr));  // L^T L L_M^{-1} x
    return run_program(v, *K4, t1, y, st, nullptr);      // L_M^{-T} L^T L L_M^{-1} x
  };
  auto applyMi = [&](double* x, double* y) -> int {
    if (which == SVAR_SPEC_LML) {
      SVAR_HIP(hipMemcpyAsync(y, x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
      return SVAR_OK;
    }
    return run_program(v, *Mi, x, y, st, nullptr);
  };
  std::vector<double> al, be;
  if (rc == SVAR_OK) {
    launch_fill(r_prev, n, 0.0, st);
    SVAR_HIP(hipMemcpyAsync(r, start, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
    rc = applyMi(r, z);
  }
  double beta = 0.0, beta_prev = 1.0;
  if (rc == SVAR_OK) rc = dot(r, z, n, part, st, &beta);
  if (rc == SVAR_OK && !(beta > 0.0)) rc = inval_msg("start vector has no component (r^T M^{-1} r <= 0)");
  if (rc == SVAR_OK) beta = std::sqrt(beta);
  for (int j = 0; rc == SVAR_OK && j < nsteps; ++j) {
    // v_j = z / beta (held in z), p = K v_j
    launch_axpby(z, z, n, 1.0 / beta - 1.0, 1.0, st);  // z *= 1/beta
    rc = applyK(z, p);
    double alpha = 0.0;
    if (rc == SVAR_OK) rc = dot(z, p, n, part, st, &alpha);
    if (rc != SVAR_OK) break;
    al.push_back(alpha);
    // p -= alpha r / beta + beta r_prev / beta_prev
    launch_axpby(p, r, n, -alpha / beta, 1.0, st);
    if (j > 0) launch_axpby(p, r_prev, n, -beta / beta_prev, 1.0, st);
    std::swap(r_prev, r);
    SVAR_HIP(hipMemcpyAsync(r, p, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
    rc = applyMi(p, z);
    double bn = 0.0;
    if (rc == SVAR_OK) rc = dot(p, z, n, part, st, &bn);
    if (rc != SVAR_OK) break;
    if (!std::isfinite(bn)) {
      rc = SVAR_E_BREAKDOWN;
      set_error("non-finite value in the Lanczos recurrence");
      break;
    }
    beta_prev = beta;
    beta = bn > 0.0 ? std::sqrt(bn) : 0.0;
    if (!(beta > 1e-300 * std::max(1.0, std::fabs(alpha)))) break;  // invariant subspace
    if (j + 1 < nsteps) be.push_back(beta);
  }
  free_all(tmp);
  SVAR_TRY(rc);
  be.resize(al.size() > 0 ? al.size() - 1 : 0);
  const std::vector<double> ev = tridiag_eigs(al, be);
  for (size_t i = 0; i < ev.size(); ++i) ritz[i] = ev[i];
  *nritz = (int32_t)ev.size();
  return SVAR_OK;
}
