// Model products, L / L^T / L_M(k) sweep steps, observation operators and vector jobs.
//
// L v, L^T v (eq. def:L) and one step of the L_M(k)^{-1}, L_M(k)^{-T} recurrences (Lemma 1:
// inside a segment z_i = v_i + M_i z_{i-1}, w_i = v_i + M_{i+1}^T w_{i+1}) are all of the form
//     out_i = in_i + alpha * M^(T) x_j
// for a list of independent (i, j) block pairs, so one kernel serves all of them; a sweep is
// k-1 launches, one per position inside the segments, each covering every segment and
// right-hand side at once (§4: the segments of L_M(k) are independent).
//
// Band models (the implicit advection-diffusion step is applied through the taps of T^{-1})
// stage the input tile plus its halo in LDS so that every HBM element is read once and the
// taps are applied from LDS.
#include "svar_impl.h"

namespace svar {

// out_j of a model job, with the job's optional addend
__device__ __forceinline__ double job_out(const MJob& J, const Bases& b, int j, double v) {
  return J.use_add ? v + b.p[J.add.base][J.add.off + j] : v;
}


static constexpr int TS = JOB_TS;  // outputs per workgroup
static constexpr int YMAX = 65535;

__device__ __forceinline__ int job_id() { return blockIdx.y + YMAX * blockIdx.z; }
static dim3 jgrid(unsigned gx, int njobs) {
  return njobs <= YMAX ? dim3(gx, njobs, 1) : dim3(gx, YMAX, (njobs + YMAX - 1) / YMAX);
}

__device__ __forceinline__ double* opnd(const Bases& b, const Operand& o) {
  return b.p[o.base] + o.off;
}

__global__ __launch_bounds__(TS) void k_mstep_band(const MJob* __restrict__ jobs,
                                                   const ModelDev* __restrict__ models, Bases b,
                                                   const int* __restrict__ skip, int njobs,
                                                   const JTile* __restrict__ tl) {
  if (skip && *skip) return;
  extern __shared__ double lds[];
  const int jid = tl ? tl[blockIdx.x].job : job_id();
  if (jid >= njobs) return;
  const MJob J = jobs[jid];
  if (SVAR_JOB_SKIPPED(b, J)) return;
  const int s = J.s;
  const int j0 = tl ? tl[blockIdx.x].first : blockIdx.x * TS;
  if (j0 >= s) return;
  const double* in = opnd(b, J.in);
  double* out = opnd(b, J.out);
  const int j = j0 + threadIdx.x;
  if (J.model < 0) {  // plain copy (first block of L, segment starts)
    if (j < s) out[j] = job_out(J, b, j, in[j]);
    return;
  }
  const ModelDev& M = models[J.model];
  const int* __restrict__ off = J.trans ? M.offT : M.off;
  const double* __restrict__ w = J.trans ? M.wT : M.w;
  const int omin = J.trans ? M.ominT : M.omin;
  const int omax = J.trans ? M.omaxT : M.omax;
  const int span = TS + omax - omin;
  const double* x = opnd(b, J.x);
  for (int t = threadIdx.x; t < span; t += TS) {
    const int gu = j0 + omin + t;
    int g = gu % s;
    if (g < 0) g += s;
    lds[t] = (M.nonperiodic && (gu < 0 || gu >= s)) ? 0.0 : x[g];
  }
  __syncthreads();
  if (j >= s) return;
  double acc = 0.0;
  const int base = threadIdx.x - omin;
  for (int tp = 0; tp < M.ntap; ++tp) acc += w[tp] * lds[base + off[tp]];
  out[j] = job_out(J, b, j, in[j] + J.alpha * acc);
}

// The same products for band models whose taps fit the window o0 .. o0 + H (the dense tap
// windows of the fused sweep): the H + 1 weights and TS + H values of x are staged in LDS and
// each thread forms its output with the taps unrolled (no offset table, no global loads in the
// tap loop).
template <int H>
__global__ __launch_bounds__(TS) void k_mstep_win(const MJob* __restrict__ jobs,
                                                  const ModelDev* __restrict__ models, Bases b,
                                                  const int* __restrict__ skip, int njobs,
                                                  const JTile* __restrict__ tl) {
  __shared__ double lw[H + 1];
  __shared__ double lx[TS + H];
  if (skip && *skip) return;
  const int jid = tl ? tl[blockIdx.x].job : job_id();
  if (jid >= njobs) return;
  const MJob J = jobs[jid];
  if (SVAR_JOB_SKIPPED(b, J)) return;
  const int s = J.s;
  const int j0 = tl ? tl[blockIdx.x].first : blockIdx.x * TS;
  if (j0 >= s) return;
  const double* in = opnd(b, J.in);
  double* out = opnd(b, J.out);
  const int j = j0 + threadIdx.x;
  if (J.model < 0) {  // plain copy (first block of L, segment starts)
    if (j < s) out[j] = job_out(J, b, j, in[j]);
    return;
  }
  const ModelDev& M = models[J.model];
  const double* __restrict__ wd = J.trans ? M.wdT : M.wd;  // H + 1 weights, offsets o0 .. o0+H
  const int o0 = J.trans ? M.wd0T : M.wd0;
  const double* x = opnd(b, J.x);
  for (int d = threadIdx.x; d <= H; d += TS) lw[d] = wd[d];
  for (int t2 = threadIdx.x; t2 < TS + H; t2 += TS) {
    int g = (j0 + o0 + t2) % s;
    if (g < 0) g += s;
    lx[t2] = x[g];
  }
  __syncthreads();
  if (j >= s) return;
  double acc = 0.0;
#pragma unroll
  for (int d = 0; d <= H; ++d) acc += lw[d] * lx[threadIdx.x + d];
  out[j] = job_out(J, b, j, in[j] + J.alpha * acc);
}

// Whole L_M(k) sweep of one segment in one workgroup (band models whose taps fit a contiguous
// window of SWEEP_H + 1 offsets, s <= SWEEP_MAXS): the running state stays in LDS (two buffers)
// for all steps of the segment, so a sweep costs one launch instead of k - 1.
//   forward  (trans = 0): z_b unchanged, z_i = v_i + M z_{i-1},     i = b+1 .. e
//   backward (trans = 1): w_e unchanged, w_i = v_i + M^T w_{i+1},   i = e-1 .. b
// in place on vec (v_i is read from vec before block i is overwritten).  Each thread computes
// SWEEP_R consecutive outputs from a register window of SWEEP_R + SWEEP_H staged values; the
// tap weights are uniform across the workgroup (scalar loads) and the tap loop is unrolled.
template <int R, int H>
__global__ __launch_bounds__(256) void k_sweep_band(const SJob* __restrict__ jobs,
                                                    const ModelDev* __restrict__ models, Bases b,
                                                    const int* __restrict__ skip, int njobs) {
  extern __shared__ double st[];  // 2 s
  if (skip && *skip) return;
  if (job_id() >= njobs) return;
  const SJob J = jobs[job_id()];
  if (SVAR_JOB_SKIPPED(b, J)) return;
  const int s = J.s;
  const ModelDev& M = models[J.model];
  const double* __restrict__ wd = J.trans ? M.wdT : M.wd;  // H + 1 weights, offsets o0 .. o0+H
  const int o0 = J.trans ? M.wd0T : M.wd0;
  double* vec = opnd(b, J.vec);
  const bool outplace = J.src.base >= 0 || J.sub.base >= 0;
  const double* src = J.src.base >= 0 ? opnd(b, J.src) : vec;
  const double* sub = J.sub.base >= 0 ? opnd(b, J.sub) : nullptr;
  double* cur = st;
  double* nxt = st + s;
  const int first = J.trans ? J.len - 1 : 0;
  for (int j = threadIdx.x; j < s; j += blockDim.x) {
    const int64_t e = (int64_t)first * s + j;
    double v = src[e];
    if (sub) v -= sub[e];
    cur[j] = v;
    if (outplace) vec[e] = v;
  }
  __syncthreads();
  for (int t = 1; t < J.len; ++t) {
    const int blk = J.trans ? J.len - 1 - t : t;
    double* row = vec + (int64_t)blk * s;
    const double* srow = src + (int64_t)blk * s;
    const double* brow = sub ? sub + (int64_t)blk * s : nullptr;
    for (int j0 = threadIdx.x * R; j0 < s; j0 += blockDim.x * R) {
      // window value m = cur[j0 + o0 + m] is loaded just before its first use (tap d = m - R + 1)
      // so only R values are live at a time
      int gb = j0 + o0;
      gb = gb < 0 ? gb + s : (gb >= s ? gb - s : gb);
      double xw[R + H];
#pragma unroll
      for (int m = 0; m < R - 1; ++m) {
        const int g = gb + m;
        xw[m] = cur[g >= s ? g - s : g];
      }
      double acc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = 0.0;
#pragma unroll
      for (int d = 0; d <= H; ++d) {
        const int g = gb + d + R - 1;
        xw[d + R - 1] = cur[g >= s ? (g >= 2 * s ? g - 2 * s : g - s) : g];
        const double wv = wd[d];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += wv * xw[r + d];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int j = j0 + r;
        if (j < s) {
          const double v = (brow ? srow[j] - brow[j] : srow[j]) + acc[r];
          row[j] = v;
          nxt[j] = v;
        }
      }
    }
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
}

// Dense model maps (distinct M_i per block): one output element per thread.
__global__ __launch_bounds__(TS) void k_mstep_dense(const MJob* __restrict__ jobs,
                                                    const ModelDev* __restrict__ models, Bases b,
                                                    const int* __restrict__ skip, int njobs) {
  if (skip && *skip) return;
  if (job_id() >= njobs) return;
  const MJob J = jobs[job_id()];
  if (SVAR_JOB_SKIPPED(b, J)) return;
  const int s = J.s;
  const int j = blockIdx.x * TS + threadIdx.x;
  if (j >= s) return;
  const double* in = opnd(b, J.in);
  double* out = opnd(b, J.out);
  if (J.model < 0) {
    out[j] = job_out(J, b, j, in[j]);
    return;
  }
  const ModelDev& M = models[J.model];
  const double* Mi = M.dense + (size_t)(J.mi - 1) * s * s;
  const double* x = opnd(b, J.x);
  double acc = 0.0;
  if (J.trans)
    for (int m = 0; m < s; ++m) acc += Mi[(size_t)m * s + j] * x[m];
  else
    for (int m = 0; m < s; ++m) acc += Mi[(size_t)j * s + m] * x[m];
  out[j] = job_out(J, b, j, in[j] + J.alpha * acc);
}

__global__ __launch_bounds__(TS) void k_gather(const HJob* __restrict__ jobs, Bases b,
                                               const int* __restrict__ skip, int njobs,
                                               const JTile* __restrict__ tl) {
  if (skip && *skip) return;
  const int jid = tl ? tl[blockIdx.x].job : job_id();
  if (jid >= njobs) return;
  const HJob J = jobs[jid];
  if (SVAR_JOB_SKIPPED(b, J)) return;
  const int r = (tl ? tl[blockIdx.x].first : blockIdx.x * TS) + threadIdx.x;
  if (r >= J.rows) return;
  const double* x = opnd(b, J.x);
  double acc = 0.0;
  for (int e = 0; e < J.width; ++e)
    acc += J.vals[(size_t)r * J.width + e] * x[J.cols[(size_t)r * J.width + e]];
  opnd(b, J.out)[r] = acc;
}

__global__ __launch_bounds__(TS) void k_scatter(const HTJob* __restrict__ jobs, Bases b,
                                                const int* __restrict__ skip, int njobs,
                                                const JTile* __restrict__ tl) {
  if (skip && *skip) return;
  const int jid = tl ? tl[blockIdx.x].job : job_id();
  if (jid >= njobs) return;
  const HTJob J = jobs[jid];
  if (SVAR_JOB_SKIPPED(b, J)) return;
  const int j = (tl ? tl[blockIdx.x].first : blockIdx.x * TS) + threadIdx.x;
  if (j >= J.s) return;
  const double* y = opnd(b, J.y);
  double acc = 0.0;
  for (int e = J.ptr[j]; e < J.ptr[j + 1]; ++e) acc += J.val[e] * y[J.idx[e]];
  opnd(b, J.out)[j] += acc;
}

__global__ __launch_bounds__(TS) void k_vec(const VJob* __restrict__ jobs, Bases b,
                                            const int* __restrict__ skip, int njobs) {
  if (skip && *skip) return;
  if (job_id() >= njobs) return;
  const VJob J = jobs[job_id()];
  if (SVAR_JOB_SKIPPED(b, J)) return;
  const double* in = opnd(b, J.in);
  double* out = opnd(b, J.out);
  const double* add = J.beta != 0.0 ? opnd(b, J.add) : nullptr;
  for (int64_t j = (int64_t)blockIdx.x * TS + threadIdx.x; j < J.len; j += (int64_t)gridDim.x * TS) {
    double v = J.scale ? in[j] * J.scale[j] : (J.alpha == 0.0 ? 0.0 : in[j] * J.alpha);
    if (add) v += J.beta * add[j];
    out[j] = v;
  }
}

// L_I^{-1}, L_I^{-T} (§2.2): z_i = v_i + z_{i-1} (forward) or w_i = v_i + w_{i+1}
// (backward) over the len time blocks of one system, one thread per spatial point (the
// accesses of a block are coalesced), input src - sub (src none: vec in place)
__global__ __launch_bounds__(TS) void k_prefix(const SJob* __restrict__ jobs, Bases b,
                                               const int* __restrict__ skip, int njobs) {
  if (skip && *skip) return;
  if (job_id() >= njobs) return;
  const SJob J = jobs[job_id()];
  if (SVAR_JOB_SKIPPED(b, J)) return;
  const int j = blockIdx.x * TS + threadIdx.x;
  if (j >= J.s) return;
  double* vec = opnd(b, J.vec);
  const double* src = J.src.base >= 0 ? opnd(b, J.src) : vec;
  const double* sub = J.sub.base >= 0 ? opnd(b, J.sub) : nullptr;
  double acc = 0.0;
  for (int t = 0; t < J.len; ++t) {
    const int i = J.trans ? J.len - 1 - t : t;
    const int64_t e = (int64_t)i * J.s + j;
    acc += sub ? src[e] - sub[e] : src[e];
    vec[e] = acc;
  }
}

__global__ void k_fill(double* x, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ void k_axpby(double* y, const double* x, int64_t n, double a, double bcoef) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + bcoef * y[i];
}

static unsigned tiles(int64_t n) { return (unsigned)((n + TS - 1) / TS); }

// tiles (nullable): the launch's flat tile list, one workgroup each; else a workgroup per
// (job, 256-output tile of the longest job), the shorter jobs' extra workgroups exiting at once
static dim3 tgrid(const JTile* tl, int ntiles, int max_len, int njobs) {
  return tl ? dim3((unsigned)ntiles) : jgrid(tiles(max_len), njobs);
}
void launch_mstep_band(const MJob* jobs, int njobs, int max_s, int max_halo,
                       const ModelDev* models, Bases b, const int* skip, hipStream_t st,
                       bool windowed, const JTile* tl, int ntiles) {
  if (njobs == 0 || (tl && ntiles == 0)) return;
  const dim3 g = tgrid(tl, ntiles, max_s, njobs);
  if (windowed) {  // every band model has a dense tap window (s >= SWEEP_H + 1)
    hipLaunchKernelGGL((k_mstep_win<SWEEP_H>), g, dim3(TS), 0, st, jobs, models, b, skip, njobs,
                       tl);
    return;
  }
  // LDS: the output tile plus the widest halo of any band model (checked at set-up)
  hipLaunchKernelGGL(k_mstep_band, g, dim3(TS), (size_t)(TS + max_halo) * sizeof(double), st,
                     jobs, models, b, skip, njobs, tl);
}
void launch_sweep_band(const SJob* jobs, int njobs, int max_s, const ModelDev* models, Bases b,
                       const int* skip, hipStream_t st) {
  if (njobs == 0) return;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_sweep_band<SWEEP_R, SWEEP_H>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(2 * SWEEP_MAXS * sizeof(double)));
    attr = true;
  }
  const int threads = 256;
  hipLaunchKernelGGL((k_sweep_band<SWEEP_R, SWEEP_H>), jgrid(1, njobs), dim3(threads),
                     (size_t)2 * max_s * sizeof(double), st, jobs, models, b, skip, njobs);
}

void launch_mstep_dense(const MJob* jobs, int njobs, int max_s, const ModelDev* models, Bases b,
                        const int* skip, hipStream_t st) {
  if (njobs == 0) return;
  hipLaunchKernelGGL(k_mstep_dense, jgrid(tiles(max_s), njobs), dim3(TS), 0, st, jobs, models, b,
                     skip, njobs);
}
void launch_prefix(const SJob* jobs, int njobs, int max_s, Bases b, const int* skip,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_prefix, jgrid(tiles(max_s), njobs), dim3(TS), 0, st, jobs, b, skip, njobs);
}
void launch_gather(const HJob* jobs, int njobs, int max_rows, Bases b, const int* skip,
                   hipStream_t st, const JTile* tl, int ntiles) {
  if (njobs == 0 || max_rows == 0 || (tl && ntiles == 0)) return;
  hipLaunchKernelGGL(k_gather, tgrid(tl, ntiles, max_rows, njobs), dim3(TS), 0, st, jobs, b, skip,
                     njobs, tl);
}
void launch_scatter(const HTJob* jobs, int njobs, int max_s, Bases b, const int* skip,
                    hipStream_t st, const JTile* tl, int ntiles) {
  if (njobs == 0 || (tl && ntiles == 0)) return;
  hipLaunchKernelGGL(k_scatter, tgrid(tl, ntiles, max_s, njobs), dim3(TS), 0, st, jobs, b, skip,
                     njobs, tl);
}
void launch_vec(const VJob* jobs, int njobs, int64_t max_len, Bases b, const int* skip,
                hipStream_t st) {
  if (njobs == 0 || max_len == 0) return;
  unsigned gx = tiles(max_len);
  if (gx > 1024) gx = 1024;
  hipLaunchKernelGGL(k_vec, jgrid(gx, njobs), dim3(TS), 0, st, jobs, b, skip, njobs);
}
void launch_fill(double* x, int64_t n, double v, hipStream_t st) {
  if (n == 0) return;
  unsigned g = tiles(n);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill, dim3(g), dim3(TS), 0, st, x, n, v);
}
void launch_axpby(double* y, const double* x, int64_t n, double a, double bcoef, hipStream_t st) {
  if (n == 0) return;
  unsigned g = tiles(n);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_axpby, dim3(g), dim3(TS), 0, st, y, x, n, a, bcoef);
}

}  // namespace svar
