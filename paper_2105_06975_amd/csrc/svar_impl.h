// Internal declarations of libsvar (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "svar.h"

struct svar_handle;

namespace svar {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
#define SVAR_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) {                                                              \
      ::svar::set_error(std::string("HIP error ") + hipGetErrorString(e_) + " at " +     \
                        __FILE__ + ":" + std::to_string(__LINE__) + " (" #call ")");     \
      return SVAR_E_HIP;                                                                 \
    }                                                                                    \
  } while (0)
inline int inval_msg(const std::string& m) {
  set_error(m);
  return SVAR_E_INVAL;
}
#define SVAR_TRY(call)          \
  do {                          \
    int st_ = (call);           \
    if (st_ != SVAR_OK) return st_; \
  } while (0)

// ------------------------------------------------------------------ addressing
// Kernels address caller and workspace vectors through a small table of base pointers
// passed by value; job tables store (base, offset) pairs so that they can be built once
// per (operation, nrhs) and reused for any caller pointers.
enum BaseId { B_IN = 0, B_OUT = 1, B_TMP = 2, B_AUX = 3 };
// flags (nullable): per-job skip flags of a solve.  Every job carries the index of the flag
// that retires it: 1 + sys for the jobs of one system (window w, rhs r: sys = w nrhs + r),
// 1 + nsys + w for the covariance products of window w (all its right-hand sides at once);
// a nonzero flag makes the job return at once (the system has converged this cycle).
struct Bases {
  double* p[4];
  const int* flags;
};
#define SVAR_JOB_SKIPPED(b, J) ((b).flags && (b).flags[(J).flag])
struct Operand {
  int32_t base;  // BaseId, or -1 for "none"
  int32_t pad;
  int64_t off;   // element offset
};

// ------------------------------------------------------------------ covariance GEMM
// Y[:, c] = beta * Z[:, c] + alpha0 * alpha[c % per] * (C X)[:, c], C an n x n matrix
// stored row-major (lda = n).  Column c of X lives at X.off + (c / per) * xo + (c % per) * xi.
enum { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };
// n rounded up to a multiple of 4 (row stride of the padded float32 matrix copies)
inline int pad4(int n) { return (n + 3) & ~3; }

struct GemmProb {
  const void* C;
  int32_t n, ncols, per, splits;
  Operand X, Y, Z;
  int64_t xo, xi, yo, yi, zo, zi;
  const double* alpha;  // [per] device, or nullptr
  double alpha0, beta;
  int64_t ws_off;       // element offset of the split-K partials (splits > 1)
  int32_t dtype, flag;  // flag: skip flag index (see Bases)
  int32_t ld, pad_ld;   // row stride of C in elements (>= n; 0 = n)
  const double* zeros;  // >= n zeros: stands in for rows / columns past the edge
};
struct GemmTask {
  int32_t prob, row0, k0, k1, col0, split;
};
// row tiles (of 16) per wave of the FP64 product, by the number of 16-column tiles
constexpr int gemm_rt(int ct) { return ct <= 5 ? 2 : 1; }

// ------------------------------------------------------------------ model products
// out[j] = in[j] + alpha * (M op x)[j], j < s, for one block; op = M_mi or M_mi^T.
struct MJob {
  Operand in, x, out;
  int32_t model, mi, trans, s;
  double alpha;
  Operand add;        // use_add: out also receives + add (band and dense models)
  int32_t use_add, flag;
};
enum ModelKind { MK_BAND = 0, MK_DENSE = 1, MK_L96 = 2 };
// one whole L_M(k) sweep segment: blocks vec.off + [0, len) s, in place
struct SJob {
  Operand vec;
  int32_t model, trans, s, len;
  // sources of the sweep's input (base -1: none): the input is src - sub (src none: vec
  // itself, in place), so a copy or a difference before the sweep needs no launch of its own
  Operand src, sub;
  int32_t flag, pad;
};
constexpr int SWEEP_MAXS = 8192;  // LDS holds two state vectors (128 KB)
constexpr int SWEEP_R = 8;        // outputs per thread of the fused sweep
constexpr int SWEEP_H = 63;       // widest contiguous tap window (offsets o0 .. o0 + SWEEP_H)
struct ModelDev {
  int32_t kind, s, N, ntap;
  const int32_t* off;    // band taps of M
  const double* w;
  const int32_t* offT;   // band taps of M^T
  const double* wT;
  int32_t omin, omax, ominT, omaxT;
  const double* wd;      // taps of M on the contiguous window o0 .. o0 + SWEEP_H (zero padded)
  const double* wdT;     // same for M^T
  int32_t wd0, wd0T;     // window starts; wd == nullptr when the taps do not fit
  const double* dense;   // N matrices, M_i at (i-1)*s*s
  // Lorenz-96 tangent linear model
  const double* traj;    // [N+1][s]
  double F, dt;
  int32_t nsteps;
  int32_t nonperiodic;   // band models: values outside 0..s-1 are zero (Dirichlet boundaries)
};

// ------------------------------------------------------------------ H
struct HJob {            // gather: out[r] = sum_w vals[r*w+e] * x[cols[r*w+e]]
  Operand x, out;
  const int32_t* cols;
  const double* vals;
  int32_t rows, width;
  int32_t flag, pad;
};
struct HTJob {           // scatter-add: out[j] += sum_{e in ptr[j]..ptr[j+1]} val[e] * y[idx[e]]
  Operand y, out;
  const int32_t* ptr;
  const int32_t* idx;
  const double* val;
  int32_t s, flag;
};
struct VJob {            // out[j] = in[j] * (scale ? scale[j] : alpha) + beta * add[j], j < len
  Operand in, out;
  const double* scale;
  double alpha;
  int64_t len;
  Operand add;            // read only when beta != 0
  double beta;
  int32_t flag, pad;
};

// ------------------------------------------------------------------ launch programs
enum LaunchKind { LK_MSTEP_BAND, LK_MSTEP_DENSE, LK_MSTEP_L96, LK_GATHER, LK_SCATTER, LK_VEC,
                  LK_GEMM, LK_SWEEP_BAND, LK_NET, LK_PREFIX };
struct GemmPlanDev {
  GemmProb* probs = nullptr;   // device
  GemmTask* tasks = nullptr;   // device
  int nprob = 0, ntask = 0, maxct = 0;
  std::vector<int> reduce_probs;  // host indices of problems with splits > 1
  int* reduce_list = nullptr;     // device copy
  int64_t max_reduce_elems = 0;
  int64_t ws_elems = 0;
  int dtype = DT_F64;
  int tiled = 0;                  // 1: LDS-tiled kernel (128-row tiles), 0: k-split kernel
  int direct = 0;                 // tiled: every matrix 4-element aligned (rows read to registers)
  int target = 512;               // workgroups the planner aims for
  std::vector<GemmProb> hprobs;   // host copy of the problems (autotuning re-plans them)
  std::string key;                // shape key of the launch (autotuning cache)
};
// one workgroup's share of a job-table launch: outputs first .. first + JOB_TS - 1 of job
// `job` (a flat list of the tiles that exist, so jobs of different lengths share a launch
// without empty workgroups)
constexpr int JOB_TS = 256;
struct JTile {
  int32_t job, first;
};
struct Launch {
  LaunchKind kind;
  void* jobs = nullptr;   // device job table
  int njobs = 0;
  const JTile* tiles = nullptr;  // model products, H and H^T: the workgroups' tiles
  int ntiles = 0;
  int grid_x = 0;
  int max_s = 0;
  GemmPlanDev gemm;
  int kclass = -1;        // timing class
};
struct Program {
  std::vector<Launch> launches;
  int64_t tmp_elems = 0;  // B_TMP workspace needed
  int64_t aux_elems = 0;  // B_AUX: the handle's shared D z1 buffer (P_I with A in float64)
  // component counters per application (Tables 4 and 5 style): M, M^T, D, R, Rhat^-1, Dhat^-1
  int64_t cnt[6] = {0, 0, 0, 0, 0, 0};
};

// kernel launchers (defined in the .hip files)
void launch_mstep_band(const MJob* jobs, int njobs, int max_s, int max_halo,
                       const ModelDev* models, Bases b, const int* skip, hipStream_t st,
                       bool windowed = false, const JTile* tiles = nullptr, int ntiles = 0);
void launch_mstep_dense(const MJob* jobs, int njobs, int max_s, const ModelDev* models,
                        Bases b, const int* skip, hipStream_t st);
void launch_sweep_band(const SJob* jobs, int njobs, int max_s, const ModelDev* models, Bases b,
                       const int* skip, hipStream_t st);
// L_I^{-1} (trans = 0: running sum over the len blocks) or L_I^{-T} (trans = 1: from the last
// block backwards) of each job's vector, input src - sub as for the sweeps
void launch_prefix(const SJob* jobs, int njobs, int max_s, Bases b, const int* skip,
                   hipStream_t st);
void launch_mstep_l96(const MJob* jobs, int njobs, int max_s, int max_steps,
                      const ModelDev* models, Bases b, const int* skip, hipStream_t st);
void launch_gather(const HJob* jobs, int njobs, int max_rows, Bases b, const int* skip,
                   hipStream_t st, const JTile* tiles = nullptr, int ntiles = 0);
void launch_scatter(const HTJob* jobs, int njobs, int max_s, Bases b, const int* skip,
                    hipStream_t st, const JTile* tiles = nullptr, int ntiles = 0);
void launch_vec(const VJob* jobs, int njobs, int64_t max_len, Bases b, const int* skip,
                hipStream_t st);
void launch_gemm(const GemmPlanDev& g, Bases b, double* ws, const int* skip, hipStream_t st);

void launch_l96_forecast(const double* x, double* y, int s, int N, double F, double h, int nsteps,
                         hipStream_t st);

// plain helpers used by set-up and drivers
void launch_fill(double* x, int64_t n, double v, hipStream_t st);
void launch_axpby(double* y, const double* x, int64_t n, double a, double b, hipStream_t st);

}  // namespace svar
