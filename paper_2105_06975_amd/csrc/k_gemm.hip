// Covariance products Y = beta Z + diag(alpha) (C X) on MFMA (gfx950).
//
// The dense covariance blocks B, Q_i = q B, R_i and the precomputed Rhat_i^{-1}, Dhat_i^{-1}
// multiply all time blocks (and right-hand sides) at once, so each product is one GEMM of an
// n x n matrix with an n x ncols panel of vectors (§6.2: "loop over the N+1 blocks" becomes
// one matrix-panel product because the blocks share the matrix).
//
// Tiling: a workgroup is four wave64s; each wave owns 16 rows of C and CT x 16 columns of the
// panel and walks its k-range in steps of 16 with v_mfma_f64_16x16x4f64.  Within a step a
// lane loads four consecutive k of its row of C and four consecutive k of its panel column,
// so both operands are read as 32-byte runs straight from global memory; the order in which
// the four MFMAs of a step consume k is the same for both operands, so the contraction is
// unchanged.  Splitting k over several workgroups gives enough waves for 256 CUs; the split
// partials are summed in a fixed order by a second kernel (deterministic results).
#include "svar_impl.h"

namespace svar {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
// global-address-space pointer: loads through it are global_load (counted by vmcnt only,
// so a wait can target the older of two in-flight batches); generic pointers become flat
// loads whose counter can only be waited to zero
typedef const __attribute__((address_space(1))) double* gdp;

__device__ __forceinline__ double* opnd(const Bases& b, const Operand& o) {
  return b.p[o.base] + o.off;
}

__device__ __forceinline__ void gemm_store(const GemmProb& P, const Bases& b, int r, int c,
                                           double acc) {
  const int co = c / P.per, ci = c - co * P.per;
  const double a = P.alpha0 * (P.alpha ? P.alpha[ci] : 1.0);
  double y = a * acc;
  if (P.Z.base >= 0 && P.beta != 0.0) y += P.beta * opnd(b, P.Z)[co * P.zo + ci * P.zi + r];
  opnd(b, P.Y)[co * P.yo + ci * P.yi + r] = y;
}

// element loads of the matrix in its storage type, widened to double / float
__device__ __forceinline__ double ld_c(const void* C, size_t i, int dt) {
  if (dt == DT_F64) return ((const double*)C)[i];
  if (dt == DT_F32) return (double)((const float*)C)[i];
  const unsigned short h = ((const unsigned short*)C)[i];
  return (double)__uint_as_float(((unsigned)h) << 16);
}

// FP64 product.  Workgroup = 4 waves sharing one (RT x 16)-row tile and its k-range: wave w
// takes the w-th quarter of the k-range, so the workgroup's partial sums are combined in LDS
// (two rounds, fixed order) and only the split-K over workgroups goes through global memory.
// Each wave keeps RT x CT accumulator tiles; the operand fragments of step s+1 are loaded
// while the MFMAs of step s run (two register buffers), which hides global-load latency.
// Operand loads are unconditional from always-valid addresses (rows / columns past the end
// are clamped to the first one) and the values are masked afterwards, so no load sits behind
// a branch and all loads of a step stay in flight together.  Full steps need no k check; the
// ragged last step clamps each k index as well.
template <int CT, int RT>
__device__ __forceinline__ void gemm_load_full(const gdp (&A)[RT], const bool (&rok)[RT],
                                               const gdp (&xp)[CT],
                                               const bool (&cok)[CT], int kk, double (&a)[RT][4],
                                               double (&bb)[CT][4]) {
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) a[rt][i] = A[rt][kk + i];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int i = 0; i < 4; ++i) bb[ct][i] = xp[ct][kk + i];
}
template <int CT, int RT>
__device__ __forceinline__ void gemm_load_tail(const gdp (&A)[RT], const bool (&rok)[RT],
                                               const gdp (&xp)[CT],
                                               const bool (&cok)[CT], int kk, int ke, int n,
                                               double (&a)[RT][4], double (&bb)[CT][4]) {
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double v = A[rt][min(kk + i, n - 1)];
      a[rt][i] = (rok[rt] && kk + i < ke) ? v : 0.0;
    }
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double v = xp[ct][min(kk + i, n - 1)];
      bb[ct][i] = (cok[ct] && kk + i < ke) ? v : 0.0;
    }
}

template <int CT, int RT>
__device__ __forceinline__ void gemm_mfma(v4d (&acc)[RT][CT], const double (&a)[RT][4],
                                          const double (&bb)[CT][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
        acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt][i], bb[ct][i], acc[rt][ct], 0, 0, 0);
}

template <int CT, int RT>
__global__ __launch_bounds__(256) void k_gemm_f64(const GemmProb* __restrict__ probs,
                                                     const GemmTask* __restrict__ tasks,
                                                     double* __restrict__ ws, Bases b,
                                                     const int* __restrict__ skip) {
  __shared__ double red[2][RT * CT * 4][64];
  if (skip && *skip) return;
  const GemmTask t = tasks[blockIdx.x];
  const GemmProb P = probs[t.prob];
  const int lane = threadIdx.x & 63;
  // wave index as a scalar: the k-range bounds below are then uniform and the loop control
  // stays on scalar branches (no exec-masked regions around the prefetch loads)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, q = lane >> 4;
  const int rbase = t.row0;
  if (rbase >= P.n) return;
  // this wave's quarter of the workgroup k-range (multiple of 16)
  const int wlen = ((t.k1 - t.k0 + 63) / 64) * 16;
  const int kb = t.k0 + wave * wlen;
  const int ke = min(t.k1, kb + wlen);
  gdp A[RT];
  bool rok[RT];
  // rows / columns past the edge read the zero buffer, so loaded values need no masking
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int row = rbase + rt * 16 + r16;
    rok[rt] = row < P.n;
    A[rt] = (gdp)(rok[rt] ? (const double*)P.C + (size_t)row * P.n : P.zeros);
  }
  const double* X = opnd(b, P.X);
  gdp xp[CT];
  bool cok[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int c = t.col0 + ct * 16 + r16;
    cok[ct] = c < P.ncols;
    const int cc = cok[ct] ? c : 0;
    const int co = cc / P.per, ci = cc - co * P.per;
    xp[ct] = (gdp)(cok[ct] ? X + co * P.xo + ci * P.xi : P.zeros);
  }
  v4d acc[RT][CT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = (v4d){0.0, 0.0, 0.0, 0.0};
  double a0[RT][4], b0[CT][4], a1[RT][4], b1[CT][4];
  // full steps of 16, the next step's fragments loaded while the current one multiplies
  const int nfull = ke > kb ? (ke - kb) >> 4 : 0;
  if (nfull > 0) gemm_load_full<CT, RT>(A, rok, xp, cok, kb + 4 * q, a0, b0);
  int s = 0;
  // sched_barrier keeps each load batch ahead of the MFMA batch that does not need it, so the
  // wait before the MFMAs covers only the older batch
  for (; s + 2 <= nfull; s += 2) {
    gemm_load_full<CT, RT>(A, rok, xp, cok, kb + 16 * (s + 1) + 4 * q, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    gemm_mfma<CT, RT>(acc, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    // unconditional prefetch (a branch here would force a full wait at the join); the last
    // trip re-loads the final full step, which is never used
    gemm_load_full<CT, RT>(A, rok, xp, cok, kb + 16 * min(s + 2, nfull - 1) + 4 * q, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    gemm_mfma<CT, RT>(acc, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (s < nfull) gemm_mfma<CT, RT>(acc, a0, b0);
  const int kt = kb + 16 * nfull;
  if (kt < ke) {  // ragged last step
    gemm_load_tail<CT, RT>(A, rok, xp, cok, kt + 4 * q, ke, P.n, a0, b0);
    gemm_mfma<CT, RT>(acc, a0, b0);
  }
  // combine the four waves: (2,3) -> (0,1), then 1 -> 0
#pragma unroll
  for (int round = 0; round < 2; ++round) {
    const int half = round == 0 ? 2 : 1;
    if (wave >= half && wave < 2 * half) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int e = 0; e < 4; ++e) red[wave - half][(rt * CT + ct) * 4 + e][lane] = acc[rt][ct][e];
    }
    __syncthreads();
    if (wave < half) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[rt][ct][e] += red[wave][(rt * CT + ct) * 4 + e][lane];
    }
    __syncthreads();
  }
  if (wave != 0) return;
  // v_mfma_f64_16x16x4f64 result layout: accumulator element e of lane (q, r16) is row
  // q + 4 e of the 16 x 16 tile (rows interleaved across the four lane groups), column r16
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int c = t.col0 + ct * 16 + r16;
    if (c >= P.ncols) continue;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rbase + rt * 16 + q + 4 * e;
        if (r >= P.n) continue;
        if (P.splits > 1)
          ws[P.ws_off + ((int64_t)t.split * P.ncols + c) * P.n + r] = acc[rt][ct][e];
        else
          gemm_store(P, b, r, c, acc[rt][ct][e]);
      }
  }
}

// Reduced-precision matrix (float32 or bfloat16 storage) with float32 MFMA accumulation.
// The panel is converted to float on load; accumulation is float32 (v_mfma_f32_16x16x4f32).
template <int CT>
__global__ __launch_bounds__(256) void k_gemm_lp(const GemmProb* __restrict__ probs,
                                                 const GemmTask* __restrict__ tasks,
                                                 double* __restrict__ ws, Bases b,
                                                 const int* __restrict__ skip) {
  if (skip && *skip) return;
  const GemmTask t = tasks[blockIdx.x];
  const GemmProb P = probs[t.prob];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, q = lane >> 4;
  const int rbase = t.row0 + wave * 16;
  if (rbase >= P.n) return;
  const int rowA = rbase + r16;
  const bool rowok = rowA < P.n;
  const size_t abase = (size_t)(rowok ? rowA : 0) * P.n;
  const double* X = opnd(b, P.X);
  const double* xp[CT];
  bool cok[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int c = t.col0 + ct * 16 + r16;
    cok[ct] = c < P.ncols;
    const int cc = cok[ct] ? c : 0;
    const int co = cc / P.per, ci = cc - co * P.per;
    xp[ct] = X + co * P.xo + ci * P.xi;
  }
  v4f acc[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) acc[ct] = (v4f){0.f, 0.f, 0.f, 0.f};
  for (int k = t.k0; k < t.k1; k += 16) {
    const int kk = k + 4 * q;
    float a[4], bb[CT][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kc = min(kk + i, P.n - 1);  // always-valid address, value masked below
      const float v = (float)ld_c(P.C, abase + kc, P.dtype);
      a[i] = (rowok && kk + i < t.k1) ? v : 0.f;
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float v = (float)xp[ct][min(kk + i, P.n - 1)];
        bb[ct][i] = (cok[ct] && kk + i < t.k1) ? v : 0.f;
      }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bb[ct][i], acc[ct], 0, 0, 0);
  }
  // v_mfma_f32_16x16x4f32 result layout: element e of lane (q, r16) is row 4 q + e
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int c = t.col0 + ct * 16 + r16;
    if (c >= P.ncols) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = rbase + 4 * q + e;
      if (r >= P.n) continue;
      if (P.splits > 1)
        ws[P.ws_off + ((int64_t)t.split * P.ncols + c) * P.n + r] = (double)acc[ct][e];
      else
        gemm_store(P, b, r, c, (double)acc[ct][e]);
    }
  }
}

__global__ __launch_bounds__(256) void k_gemm_reduce(const GemmProb* __restrict__ probs,
                                                     const int* __restrict__ list,
                                                     const double* __restrict__ ws, Bases b,
                                                     const int* __restrict__ skip) {
  if (skip && *skip) return;
  const GemmProb P = probs[list[blockIdx.y]];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t tot = (int64_t)P.n * P.ncols;
  if (e >= tot) return;
  const int c = (int)(e / P.n), r = (int)(e - (int64_t)c * P.n);
  double s = 0.0;
  for (int sp = 0; sp < P.splits; ++sp) s += ws[P.ws_off + ((int64_t)sp * P.ncols + c) * P.n + r];
  gemm_store(P, b, r, c, s);
}

template <int CT>
static void launch_ct(const GemmPlanDev& g, Bases b, double* ws, const int* skip,
                      hipStream_t st) {
  if (g.dtype == DT_F64)
    hipLaunchKernelGGL((k_gemm_f64<CT, gemm_rt(CT)>), dim3(g.ntask), dim3(256), 0, st, g.probs,
                       g.tasks, ws, b, skip);
  else
    hipLaunchKernelGGL(k_gemm_lp<CT>, dim3(g.ntask), dim3(256), 0, st, g.probs, g.tasks, ws, b,
                       skip);
}

void launch_gemm(const GemmPlanDev& g, Bases b, double* ws, const int* skip, hipStream_t st) {
  if (g.ntask == 0) return;
  switch (g.maxct) {
    case 1: launch_ct<1>(g, b, ws, skip, st); break;
    case 2: launch_ct<2>(g, b, ws, skip, st); break;
    case 3: launch_ct<3>(g, b, ws, skip, st); break;
    case 4: launch_ct<4>(g, b, ws, skip, st); break;
    case 5: launch_ct<5>(g, b, ws, skip, st); break;
    case 6: launch_ct<6>(g, b, ws, skip, st); break;
    case 7: launch_ct<7>(g, b, ws, skip, st); break;
    default: launch_ct<8>(g, b, ws, skip, st); break;
  }
  if (!g.reduce_probs.empty()) {
    const int gx = (int)((g.max_reduce_elems + 255) / 256);
    hipLaunchKernelGGL(k_gemm_reduce, dim3(gx, (unsigned)g.reduce_probs.size()), dim3(256), 0, st,
                       g.probs, g.reduce_list, ws, b, skip);
  }
}

}  // namespace svar
