// Preconditioned MINRES driver (internal).
#pragma once
#include "svar_handle.h"

namespace svar {
int solve_minres(svar_handle* h, const svar_solve_opts* o, int nrhs, const double* rhs, double* x,
                 svar_solve_info* info, hipStream_t st);
}  // namespace svar
