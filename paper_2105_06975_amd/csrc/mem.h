// Device allocation helpers (internal).
#pragma once
#include "svar_impl.h"

namespace svar {

template <class T>
inline int dalloc(std::vector<void*>& owner, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed: " +
              hipGetErrorString(e));
    *p = nullptr;
    return SVAR_E_NOMEM;
  }
  owner.push_back((void*)*p);
  return SVAR_OK;
}
template <class T>
inline int upload(std::vector<void*>& owner, T** p, const T* src, size_t count, hipStream_t st) {
  SVAR_TRY(dalloc(owner, p, count));
  if (count) SVAR_HIP(hipMemcpyAsync(*p, src, count * sizeof(T), hipMemcpyHostToDevice, st));
  return SVAR_OK;
}
inline void free_all(std::vector<void*>& v) {
  for (void* p : v) (void)hipFree(p);
  v.clear();
}

// defined in svar_api.hip
int get_program(svar_handle* h, int op, int nrhs, int prec, Program** out, hipStream_t st);
// skip: every launch returns at once when *skip != 0; flags: per-job skip flags (see Bases)
int run_program(svar_handle* h, const Program& P, double* in, double* out, hipStream_t st,
                const int* skip, const int* flags = nullptr);
int64_t handle_total(const svar_handle* h, int nrhs);
int64_t state_total(const svar_handle* h, int nrhs);
bool timing_any(const svar_handle* h);
void timed_begin(svar_handle* h, int kc, hipStream_t st, hipEvent_t* e0, hipEvent_t* e1);
void timed_end(svar_handle* h, int kc, hipStream_t st, hipEvent_t e0, hipEvent_t e1);
int ensure_krylov(svar_handle* h, int nrhs, int m, hipStream_t st);
// a handle over windows [w0, w1) of h sharing its matrices (created on first use, owned by h)
int get_view(svar_handle* h, int w0, int w1, svar_handle** out);
int sys_norm2(svar_handle* h, const double* x, std::vector<double>& out, hipStream_t st);

}  // namespace svar
