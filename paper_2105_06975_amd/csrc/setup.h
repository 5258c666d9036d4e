// Set-up kernel launchers (internal).
#pragma once
#include "svar_impl.h"

namespace svar {
void su_scaled_identity(double* X, int n, double a, hipStream_t st);
int su_ns_residual(double* T, int n, double* part, hipStream_t st);
void su_rowabs(const double* A, int n, double* out, hipStream_t st);
void su_symmetrize(double* X, int n, hipStream_t st);
void su_copy_scale_shift(const double* A, double* X, int n, double a, double d, hipStream_t st);
void su_scale(double* X, int64_t len, double a, hipStream_t st);
int su_sqdiff_part(const double* X, const double* Y, int64_t len, double* part, hipStream_t st);
int su_dot_part(const double* a, const double* b, int64_t len, double* part, hipStream_t st);
void su_rownorm2(const double* M, int n, double* out, hipStream_t st);
void su_row_scaled(const double* M, int n, int row, double a, double* v, hipStream_t st);
void su_rank1(double* X, int n, const double* v, double c, hipStream_t st);
void su_diag_inv(const double* R, int n, double* out, hipStream_t st);
void su_tridiag_inv_col(double a, double b, double c, int s, double* g, double* work,
                        hipStream_t st);
void su_to_f32(const double* src, void* dst, int64_t len, hipStream_t st);
void su_to_bf16(const double* src, void* dst, int64_t len, hipStream_t st);
// float32 copy of an n x n matrix with rows padded to ld >= n elements (zeros)
void su_to_f32_pad(const double* src, void* dst, int n, int ld, hipStream_t st);
// scaled Frobenius norms of the super-diagonal blocks of R (block starts pst, device)
void su_superdiag_norms(const double* R, int n, const int* pst, int npairs, double* out,
                        hipStream_t st);
}  // namespace svar
