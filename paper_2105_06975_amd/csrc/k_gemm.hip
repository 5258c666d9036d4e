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


// FP64 product.  Workgroup = 4 waves sharing one (RT x 16)-row tile and its k-range: wave w
// takes the w-th quarter of the k-range, so the workgroup's partial sums are combined in LDS
// (two rounds, fixed order) and only the split-K over workgroups goes through global memory.
// Each wave keeps RT x CT accumulator tiles; the operand fragments of step s+1 are loaded
// while the MFMAs of step s run (two register buffers), which hides global-load latency.
// Operand loads are unconditional from always-valid addresses (rows / columns past the end
// read a zero buffer) so no load sits behind a branch and all loads of a step stay in flight
// together.  Full steps need no k check; the ragged last step clamps each k index.
//
// One template serves three storage types of the matrix: double (float64 MFMA,
// v_mfma_f64_16x16x4f64), float and bfloat16 (float32 MFMA, v_mfma_f32_16x16x4f32, panel
// converted to float on load, float32 accumulation).
template <typename CS> struct gptr_of { typedef const __attribute__((address_space(1))) CS* type; };

__device__ __forceinline__ double to_acc(double v, double) { return v; }
__device__ __forceinline__ float to_acc(double v, float) { return (float)v; }
__device__ __forceinline__ float to_acc(float v, float) { return v; }
__device__ __forceinline__ float to_acc(unsigned short h, float) {
  return __uint_as_float(((unsigned)h) << 16);
}

template <typename AT> struct mfma_of;
template <> struct mfma_of<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ v4d op(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // v_mfma_f64_16x16x4f64: element e of lane group q holds row q + 4 e of the tile
  static __device__ __forceinline__ int row(int q, int e) { return q + 4 * e; }
};
template <> struct mfma_of<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ v4f op(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // v_mfma_f32_16x16x4f32: element e of lane group q holds row 4 q + e of the tile
  static __device__ __forceinline__ int row(int q, int e) { return 4 * q + e; }
};

template <int CT, int RT, typename CS, typename AT>
__device__ __forceinline__ void gemm_load_full(const typename gptr_of<CS>::type (&A)[RT],
                                               const gdp (&xp)[CT], int kk, AT (&a)[RT][4],
                                               AT (&bb)[CT][4]) {
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) a[rt][i] = to_acc(A[rt][kk + i], AT());
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int i = 0; i < 4; ++i) bb[ct][i] = to_acc(xp[ct][kk + i], AT());
}
template <int CT, int RT, typename CS, typename AT>
__device__ __forceinline__ void gemm_load_tail(const typename gptr_of<CS>::type (&A)[RT],
                                               const gdp (&xp)[CT], int kk, int ke, int n,
                                               AT (&a)[RT][4], AT (&bb)[CT][4]) {
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const AT v = to_acc(A[rt][min(kk + i, n - 1)], AT());
      a[rt][i] = kk + i < ke ? v : AT(0);
    }
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const AT v = to_acc(xp[ct][min(kk + i, n - 1)], AT());
      bb[ct][i] = kk + i < ke ? v : AT(0);
    }
}

template <int CT, int RT, typename AT>
__device__ __forceinline__ void gemm_mfma(typename mfma_of<AT>::acc_t (&acc)[RT][CT],
                                          const AT (&a)[RT][4], const AT (&bb)[CT][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
        acc[rt][ct] = mfma_of<AT>::op(a[rt][i], bb[ct][i], acc[rt][ct]);
}

// Workgroup = 4 waves sharing one (RT x 16)-row tile and its k-range: wave w takes the w-th
// quarter, the four partial sums are combined in LDS (two rounds, fixed order) and only the
// split-K over workgroups goes through global memory.  The next step's fragments are loaded
// while the current step multiplies (two register buffers); scheduling barriers keep the
// batches apart so that each wait covers only the older batch.
template <int CT, int RT, typename CS, typename AT>
__global__ __launch_bounds__(256) void k_gemm(const GemmProb* __restrict__ probs,
                                              const GemmTask* __restrict__ tasks,
                                              double* __restrict__ ws, Bases b,
                                              const int* __restrict__ skip) {
  typedef typename mfma_of<AT>::acc_t acc_t;
  typedef typename gptr_of<CS>::type cptr;
  __shared__ AT red[2][RT * CT * 4][64];
  if (skip && *skip) return;
  const GemmTask t = tasks[blockIdx.x];
  const GemmProb P = probs[t.prob];
  if (SVAR_JOB_SKIPPED(b, P)) return;
  const int lane = threadIdx.x & 63;
  // wave index as a scalar: the k-range bounds are then uniform and the loop control stays on
  // scalar branches (no exec-masked regions around the prefetch loads)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, q = lane >> 4;
  const int rbase = t.row0;
  if (rbase >= P.n) return;
  const int wlen = ((t.k1 - t.k0 + 63) / 64) * 16;
  const int kb = t.k0 + wave * wlen;
  const int ke = min(t.k1, kb + wlen);
  cptr A[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int row = rbase + rt * 16 + r16;
    A[rt] = (cptr)(row < P.n ? (const CS*)P.C + (size_t)row * P.ld : (const CS*)P.zeros);
  }
  const double* X = opnd(b, P.X);
  gdp xp[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int c = t.col0 + ct * 16 + r16;
    const bool ok = c < P.ncols;
    const int cc = ok ? c : 0;
    const int co = cc / P.per, ci = cc - co * P.per;
    xp[ct] = (gdp)(ok ? X + co * P.xo + ci * P.xi : P.zeros);
  }
  acc_t acc[RT][CT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = acc_t{};
  AT a0[RT][4], b0[CT][4], a1[RT][4], b1[CT][4];
  const int nfull = ke > kb ? (ke - kb) >> 4 : 0;
  if (nfull > 0) gemm_load_full<CT, RT, CS, AT>(A, xp, kb + 4 * q, a0, b0);
  int s = 0;
  for (; s + 2 <= nfull; s += 2) {
    gemm_load_full<CT, RT, CS, AT>(A, xp, kb + 16 * (s + 1) + 4 * q, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    gemm_mfma<CT, RT, AT>(acc, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    // unconditional prefetch (a branch here would force a full wait at the join); the last
    // trip re-loads the final full step, which is never used
    gemm_load_full<CT, RT, CS, AT>(A, xp, kb + 16 * min(s + 2, nfull - 1) + 4 * q, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    gemm_mfma<CT, RT, AT>(acc, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (s < nfull) gemm_mfma<CT, RT, AT>(acc, a0, b0);
  const int kt = kb + 16 * nfull;
  if (kt < ke) {  // ragged last step
    gemm_load_tail<CT, RT, CS, AT>(A, xp, kt + 4 * q, ke, P.n, a0, b0);
    gemm_mfma<CT, RT, AT>(acc, a0, b0);
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
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int c = t.col0 + ct * 16 + r16;
    if (c >= P.ncols) continue;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rbase + rt * 16 + mfma_of<AT>::row(q, e);
        if (r >= P.n) continue;
        const double v = (double)acc[rt][ct][e];
        if (P.splits > 1)
          ws[P.ws_off + ((int64_t)t.split * P.ncols + c) * P.n + r] = v;
        else
          gemm_store(P, b, r, c, v);
      }
  }
}

__global__ __launch_bounds__(256) void k_gemm_reduce(const GemmProb* __restrict__ probs,
                                                     const int* __restrict__ list,
                                                     const double* __restrict__ ws, Bases b,
                                                     const int* __restrict__ skip) {
  if (skip && *skip) return;
  const GemmProb P = probs[list[blockIdx.y]];
  if (SVAR_JOB_SKIPPED(b, P)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t tot = (int64_t)P.n * P.ncols;
  if (e >= tot) return;
  const int c = (int)(e / P.n), r = (int)(e - (int64_t)c * P.n);
  double s = 0.0;
  for (int sp = 0; sp < P.splits; ++sp) s += ws[P.ws_off + ((int64_t)sp * P.ncols + c) * P.n + r];
  gemm_store(P, b, r, c, s);
}

// LDS-tiled product for panels of 32 or more columns.  A workgroup owns a 128-row x (16 CT)-
// column tile and a k-range; its four waves split the rows (32 each: 2 x CT accumulator
// tiles), so every staged panel element feeds 128 rows instead of 16-32, which cuts the
// panel re-reads of wide (batched) panels four- to eight-fold.  Only the panel goes through
// LDS: each 16-wide k-stage of the panel columns is loaded with consecutive lanes on
// consecutive addresses (16 lanes per 128-byte column run), converted to the accumulation
// type and stored in LDS (column stride 17 elements: the 16 columns read by a lane group hit
// distinct banks); the next stage's loads are in flight while the MFMAs consume the current
// stage (two LDS buffers, one barrier per stage).  The matrix rows belong to one wave each,
// so a wave reads them straight into registers: within a stage lane group q takes the four
// consecutive k = 4q..4q+3 (one 4-element vector load per row tile) and sub-step i of the
// MFMAs consumes k = 4q + i of both operands, the same k for matrix and panel.
template <typename CS> struct vec4_of {
  typedef CS raw __attribute__((ext_vector_type(4)));
  typedef const __attribute__((address_space(1))) raw* ptr;
};

template <int CT, typename CS, typename AT>
__global__ __launch_bounds__(256, 2) void k_gemm_tiled(const GemmProb* __restrict__ probs,
                                                    const GemmTask* __restrict__ tasks,
                                                    double* __restrict__ ws, Bases b,
                                                    const int* __restrict__ skip) {
  constexpr int KT = 16, NT = 16 * CT, AS = KT + 1;
  typedef typename mfma_of<AT>::acc_t acc_t;
  typedef typename gptr_of<CS>::type cptr;
  typedef typename vec4_of<CS>::raw craw4;
  typedef typename vec4_of<CS>::ptr cptr4;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  AT* Xs = (AT*)lds_raw;  // [2][NT * AS]
  if (skip && *skip) return;
  const GemmTask t = tasks[blockIdx.x];
  const GemmProb P = probs[t.prob];
  if (SVAR_JOB_SKIPPED(b, P)) return;
  const int tid = threadIdx.x, lane = tid & 63, r16 = lane & 15, q = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // panel loader role: k offset kl, column rsub + 16 j
  const int kl = tid & 15, rsub = tid >> 4;
  cptr arow[2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    const int row = t.row0 + wave * 32 + rt * 16 + r16;
    arow[rt] = (cptr)(row < P.n ? (const CS*)P.C + (size_t)row * P.ld : (const CS*)P.zeros);
  }
  // 4-element loads need 4-aligned rows; the k-ranges start on multiples of 64
  const bool avec = (P.ld & 3) == 0 && ((uintptr_t)P.C & (4 * sizeof(CS) - 1)) == 0;
  const double* X = opnd(b, P.X);
  gdp xcol[CT];
#pragma unroll
  for (int j = 0; j < CT; ++j) {
    const int c = t.col0 + rsub + 16 * j;
    const bool ok = c < P.ncols;
    const int cc = ok ? c : 0;
    const int co = cc / P.per, ci = cc - co * P.per;
    xcol[j] = (gdp)(ok ? X + co * P.xo + ci * P.xi : P.zeros);
  }
  acc_t acc[2][CT];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = acc_t{};
  const int nst = (t.k1 - t.k0 + KT - 1) / KT;
  craw4 ra[2];
  double rx[CT];
  bool okk = false;
  auto gload = [&](int s) {
    const int k = t.k0 + s * KT + kl;
    okk = k < t.k1;
    const int kc = okk ? k : t.k0;
#pragma unroll
    for (int j = 0; j < CT; ++j) rx[j] = xcol[j][kc];
    const int ka = t.k0 + s * KT + 4 * q;
    if (avec && ka + 4 <= t.k1) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) ra[rt] = *(cptr4)(arow[rt] + ka);
    } else {  // ragged last stage or unaligned rows: element loads, zero past the k-range
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const CS v = arow[rt][min(ka + i, t.k1 - 1)];
          ra[rt][i] = ka + i < t.k1 ? v : CS(0);
        }
    }
  };
  auto sstore = [&](int buf) {
    AT* x = Xs + buf * NT * AS;
#pragma unroll
    for (int j = 0; j < CT; ++j) x[(rsub + 16 * j) * AS + kl] = okk ? to_acc(rx[j], AT()) : AT(0);
  };
  AT av[2][4];
  auto aconv = [&]() {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) av[rt][i] = to_acc(ra[rt][i], AT());
  };
  if (nst > 0) {
    gload(0);
    sstore(0);
    aconv();
  }
  __syncthreads();
  for (int s = 0; s < nst; ++s) {
    const int buf = s & 1;
    if (s + 1 < nst) gload(s + 1);
    __builtin_amdgcn_sched_barrier(0);
    const AT* x = Xs + buf * NT * AS + r16 * AS + 4 * q;
    // raised wave priority while this wave issues its MFMAs, so that the other wave of the
    // SIMD, busy with its stores and the barrier, does not take issue slots from them
    // (C2 D product 337 -> 333 us)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int sub = 0; sub < 4; ++sub) {
      AT bv[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) bv[ct] = x[ct * 16 * AS + sub];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
          acc[rt][ct] = mfma_of<AT>::op(av[rt][sub], bv[ct], acc[rt][ct]);
      // keep each sub-step's LDS reads next to its MFMAs (fewer live registers: two waves
      // per SIMD fit, which hides the LDS latency and the stage barrier)
      __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_s_setprio(0);
    __builtin_amdgcn_sched_barrier(0);
    if (s + 1 < nst) {
      sstore(buf ^ 1);
      aconv();
    }
    __syncthreads();
  }
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int c = t.col0 + ct * 16 + r16;
    if (c >= P.ncols) continue;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = t.row0 + wave * 32 + rt * 16 + mfma_of<AT>::row(q, e);
        if (r >= P.n) continue;
        const double v = (double)acc[rt][ct][e];
        if (P.splits > 1)
          ws[P.ws_off + ((int64_t)t.split * P.ncols + c) * P.n + r] = v;
        else
          gemm_store(P, b, r, c, v);
      }
  }
}

// The same product with the matrix rows staged in LDS as well (16 lanes per 128-byte row run,
// stride 17): used when a matrix's rows are not 4-element aligned (n not a multiple of 4), where
// the register path above would fall back to single-element loads spread over 16 rows.
template <int CT, typename CS, typename AT>
__global__ __launch_bounds__(256, 2) void k_gemm_tiled_lds(const GemmProb* __restrict__ probs,
                                                    const GemmTask* __restrict__ tasks,
                                                    double* __restrict__ ws, Bases b,
                                                    const int* __restrict__ skip) {
  constexpr int KT = 16, MT = 128, NT = 16 * CT, AS = KT + 1;
  typedef typename mfma_of<AT>::acc_t acc_t;
  typedef typename gptr_of<CS>::type cptr;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  AT* As = (AT*)lds_raw;             // [2][MT * AS]
  AT* Xs = As + 2 * MT * AS;         // [2][NT * AS]
  if (skip && *skip) return;
  const GemmTask t = tasks[blockIdx.x];
  const GemmProb P = probs[t.prob];
  if (SVAR_JOB_SKIPPED(b, P)) return;
  const int tid = threadIdx.x, lane = tid & 63, r16 = lane & 15, q = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // loader role: k offset kl, row / column rsub + 16 j
  const int kl = tid & 15, rsub = tid >> 4;
  cptr arow[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int row = t.row0 + rsub + 16 * j;
    arow[j] = (cptr)(row < P.n ? (const CS*)P.C + (size_t)row * P.ld : (const CS*)P.zeros);
  }
  const double* X = opnd(b, P.X);
  gdp xcol[CT];
#pragma unroll
  for (int j = 0; j < CT; ++j) {
    const int c = t.col0 + rsub + 16 * j;
    const bool ok = c < P.ncols;
    const int cc = ok ? c : 0;
    const int co = cc / P.per, ci = cc - co * P.per;
    xcol[j] = (gdp)(ok ? X + co * P.xo + ci * P.xi : P.zeros);
  }
  acc_t acc[2][CT];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = acc_t{};
  const int nst = (t.k1 - t.k0 + KT - 1) / KT;
  CS ra[8];
  double rx[CT];
  bool okk = false;
  auto gload = [&](int s) {
    const int k = t.k0 + s * KT + kl;
    okk = k < t.k1;
    const int kc = okk ? k : t.k0;
#pragma unroll
    for (int j = 0; j < 8; ++j) ra[j] = arow[j][kc];
#pragma unroll
    for (int j = 0; j < CT; ++j) rx[j] = xcol[j][kc];
  };
  auto sstore = [&](int buf) {
    AT* a = As + buf * MT * AS;
    AT* x = Xs + buf * NT * AS;
#pragma unroll
    for (int j = 0; j < 8; ++j) a[(rsub + 16 * j) * AS + kl] = okk ? to_acc(ra[j], AT()) : AT(0);
#pragma unroll
    for (int j = 0; j < CT; ++j) x[(rsub + 16 * j) * AS + kl] = okk ? to_acc(rx[j], AT()) : AT(0);
  };
  if (nst > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  for (int s = 0; s < nst; ++s) {
    const int buf = s & 1;
    if (s + 1 < nst) gload(s + 1);
    __builtin_amdgcn_sched_barrier(0);
    const AT* a = As + buf * MT * AS + (wave * 32 + r16) * AS;
    const AT* x = Xs + buf * NT * AS + r16 * AS;
#pragma unroll
    for (int sub = 0; sub < 4; ++sub) {
      const int kk = 4 * sub + q;
      AT av[2], bv[CT];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) av[rt] = a[rt * 16 * AS + kk];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) bv[ct] = x[ct * 16 * AS + kk];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = mfma_of<AT>::op(av[rt], bv[ct], acc[rt][ct]);
      // keep each sub-step's LDS reads next to its MFMAs (fewer live registers: two waves
      // per SIMD fit, which hides the LDS latency and the stage barrier)
      __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (s + 1 < nst) sstore(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int c = t.col0 + ct * 16 + r16;
    if (c >= P.ncols) continue;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = t.row0 + wave * 32 + rt * 16 + mfma_of<AT>::row(q, e);
        if (r >= P.n) continue;
        const double v = (double)acc[rt][ct][e];
        if (P.splits > 1)
          ws[P.ws_off + ((int64_t)t.split * P.ncols + c) * P.n + r] = v;
        else
          gemm_store(P, b, r, c, v);
      }
  }
}

template <int CT, typename CS, typename AT>
static void launch_tiled_t(const GemmPlanDev& g, Bases b, double* ws, const int* skip,
                           hipStream_t st) {
  if (g.direct) {
    const size_t lds = (size_t)2 * (16 * CT) * 17 * sizeof(AT);
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute((const void*)k_gemm_tiled<CT, CS, AT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      attr = true;
    }
    hipLaunchKernelGGL((k_gemm_tiled<CT, CS, AT>), dim3(g.ntask), dim3(256), lds, st, g.probs,
                       g.tasks, ws, b, skip);
    return;
  }
  const size_t lds = (size_t)2 * (128 + 16 * CT) * 17 * sizeof(AT);
  static bool attr_lds = false;
  if (!attr_lds) {
    (void)hipFuncSetAttribute((const void*)k_gemm_tiled_lds<CT, CS, AT>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr_lds = true;
  }
  hipLaunchKernelGGL((k_gemm_tiled_lds<CT, CS, AT>), dim3(g.ntask), dim3(256), lds, st, g.probs,
                     g.tasks, ws, b, skip);
}
template <int CT>
static void launch_tiled(const GemmPlanDev& g, Bases b, double* ws, const int* skip,
                         hipStream_t st) {
  if (g.dtype == DT_F64)
    launch_tiled_t<CT, double, double>(g, b, ws, skip, st);
  else if (g.dtype == DT_F32)
    launch_tiled_t<CT, float, float>(g, b, ws, skip, st);
  else
    launch_tiled_t<CT, unsigned short, float>(g, b, ws, skip, st);
}

template <int CT>
static void launch_ct(const GemmPlanDev& g, Bases b, double* ws, const int* skip,
                      hipStream_t st) {
  constexpr int RT = gemm_rt(CT);
  if (g.dtype == DT_F64)
    hipLaunchKernelGGL((k_gemm<CT, RT, double, double>), dim3(g.ntask), dim3(256), 0, st, g.probs,
                       g.tasks, ws, b, skip);
  else if (g.dtype == DT_F32)
    hipLaunchKernelGGL((k_gemm<CT, RT, float, float>), dim3(g.ntask), dim3(256), 0, st, g.probs,
                       g.tasks, ws, b, skip);
  else
    hipLaunchKernelGGL((k_gemm<CT, RT, unsigned short, float>), dim3(g.ntask), dim3(256), 0, st,
                       g.probs, g.tasks, ws, b, skip);
}

void launch_gemm(const GemmPlanDev& g, Bases b, double* ws, const int* skip, hipStream_t st) {
  if (g.ntask == 0) return;
  if (g.tiled) {
    switch (g.maxct) {
      case 2: launch_tiled<2>(g, b, ws, skip, st); break;
      case 3: launch_tiled<3>(g, b, ws, skip, st); break;
      case 4: launch_tiled<4>(g, b, ws, skip, st); break;
      case 5: launch_tiled<5>(g, b, ws, skip, st); break;
      case 6: launch_tiled<6>(g, b, ws, skip, st); break;
      case 7: launch_tiled<7>(g, b, ws, skip, st); break;
      case 8: launch_tiled<8>(g, b, ws, skip, st); break;
      default: launch_tiled<9>(g, b, ws, skip, st); break;
    }
  } else switch (g.maxct) {
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
