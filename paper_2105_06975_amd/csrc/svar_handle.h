// Handle state of libsvar (internal).
#pragma once
#include <array>
#include <memory>

#include "krylov.h"
#include "net.h"
#include "svar_impl.h"

struct svar_handle;

namespace svar {

struct WinDev {
  int s = 0, N = 0, nb = 0, P = 0;
  int64_t n = 0;                     // saddle length per right-hand side
  std::vector<int> p, poff;          // per block, offsets inside the obs component
  // D
  std::vector<double*> dmats;        // device, s x s
  std::vector<int> d_index;
  std::vector<double> d_scale;
  double* d_scale_dev = nullptr;     // [nb]
  double* neg_d_scale_dev = nullptr; // [nb], -d_scale
  // R
  std::vector<double*> rmats;        // device, p x p
  std::vector<int> rmat_p;
  std::vector<int> r_index;
  // Rhat^{-1} per distinct R: dense inverse or inverse diagonal
  std::vector<double*> rhat_inv;
  std::vector<double*> rhat_dinv;
  double* rhat_dinv_blocks = nullptr; // [P] inverse diagonal laid out per block (DIAG)
  std::vector<double> rr_gamma, me_T, lam1;
  // R_block (Alg. 3): per distinct R, the groups (first row, end row, element offset of the
  // group's inverse inside rhat_inv[m]); rhat_inv_elems: doubles held by rhat_inv[m]
  std::vector<std::vector<std::array<int64_t, 3>>> rblk;
  std::vector<int64_t> rhat_inv_elems;
  // Dhat^{-1}: distinct inverses and the one used by each block
  std::vector<double*> dhat_inv;
  std::vector<int> dhat_of_block;
  // low-precision copies for the mixed paths (per distinct matrix)
  std::vector<void*> dmats_f32, rmats_f32, dmats_bf16, rhat_inv_bf16, dhat_inv_bf16;
  std::vector<void*> rhat_inv_f32, dhat_inv_f32;
  // H (ELL) and its transpose (CSR per block)
  int hw = 1;
  int32_t* h_cols = nullptr;
  double* h_vals = nullptr;
  std::vector<int64_t> h_off;        // per block, entry offset
  int32_t* ht_ptr = nullptr;         // nb x (s+1)
  int32_t* ht_idx = nullptr;
  double* ht_val = nullptr;
  std::vector<int64_t> ht_ent_off;   // per block, entry offset
  // model
  int model_id = 0;
  int model_kind = MK_BAND;
};

struct ProgKey {
  int op, nrhs, prec;  // op code, rhs count, precision variant
  bool operator<(const ProgKey& o) const {
    if (op != o.op) return op < o.op;
    if (nrhs != o.nrhs) return nrhs < o.nrhs;
    return prec < o.prec;
  }
};

// internal program codes (beyond the public SVAR_OP_*)
// PROG_PD / PROG_AD: P_I that also leaves D z1 (float64) in the handle's dz1 buffer, and the
// A that adds that buffer instead of forming D z1 again (A is applied to z = P u right after)
enum { PROG_A = 100, PROG_P = 101, PROG_HARVEST = 102, PROG_PD = 103, PROG_AD = 104 };
// precision variants of a program
// launch-program precisions: PV_F32 float32 covariances in A; PV_BF16P / PV_F32P bfloat16 /
// float32 covariances in P (D z1 of P_I stays float64); PV_F32ALL float32 everywhere in P
enum { PV_F64 = 0, PV_F32 = 1, PV_BF16P = 2, PV_F32P = 3, PV_F32ALL = 4 };
// program variants of the inner A and P of a SVAR_PRECISION_* setting
inline bool prec_valid(int p) {
  return p >= SVAR_PRECISION_FP64 && p <= SVAR_PRECISION_MIXED_F32;
}
inline bool prec_a64(int p) {
  return p == SVAR_PRECISION_FP64 || p == SVAR_PRECISION_FP64_F32P ||
         p == SVAR_PRECISION_FP64_BF16P;
}
inline int prec_pv_p(int p) {
  if (p == SVAR_PRECISION_MIXED_BF16P || p == SVAR_PRECISION_FP64_BF16P) return PV_BF16P;
  if (p == SVAR_PRECISION_FP64_F32P || p == SVAR_PRECISION_MIXED_F32) return PV_F32P;
  return PV_F64;
}

struct Timer {
  bool on = false;
  double total_ms = 0.0;
  int64_t launches = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
};

}  // namespace svar

struct svar_handle {
  int device = 0;
  svar_prec_opts popts{};
  std::vector<int> rb_pvec;  // copy of popts.rb_pvec (popts.rb_pvec is cleared)
  std::vector<svar::WinDev> wins;
  std::vector<svar::ModelDev> models;       // host copy
  svar::ModelDev* models_dev = nullptr;
  int max_halo = 0;
  int l96_max_steps = 0;  // largest RK4 step count of the Lorenz-96 models (LDS of their kernel)
  bool band_window = true;  // every band model has a dense tap window (windowed M-step kernel)
  std::vector<void*> allocs;                // every device allocation owned by the handle
  std::map<svar::ProgKey, svar::Program> progs;
  // workspaces
  double* gemm_ws = nullptr;
  int64_t gemm_ws_elems = 0;
  double* tmp = nullptr;
  int64_t tmp_elems = 0;
  double* dz1 = nullptr;  // D z1 of the last PROG_PD application (state layout)
  int64_t dz1_elems = 0;
  double* zeros = nullptr;       // zero-filled, at least the largest matrix order
  int64_t zeros_elems = 0;
  svar::Timer timers[SVAR_KCLASS_COUNT];
  // learned correction of the Lhat^{-T} sweep
  svar_net* net = nullptr;
  const int* net_off = nullptr;   // per-system switch-off flags during a solve (device) or NULL
  std::vector<std::unique_ptr<svar::NetApp>> netapps;
  void* net_ws = nullptr;         // activations of the in-place application
  int64_t net_ws_bytes = 0;
  int prog_gen = 0;               // bumped when cached programs are dropped
  // autotuned GEMM plans: shape key -> (tiled kernel, target workgroups)
  std::map<std::string, std::pair<int, int>> tune;
  // captured FGMRES step chunk (see fgmres_cycle)
  struct StepGraph {
    hipGraphExec_t exec = nullptr;
    hipStream_t ps = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int nrhs = -1, m = -1, gen = -1, kgen = -1, patience = 0;
    const void* pa = nullptr;
    const void* pp = nullptr;
    const int* net_off = nullptr;
    const void* bufs[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // workspaces
    double drop = 0.0;
  } graph;
  // wave scheduling: svar_solve over more systems than one Krylov workspace holds runs the
  // windows in contiguous waves, each through a view (a handle over a window range that shares
  // the parent's matrices, model tables and zero buffer, and builds its own launch programs);
  // the views carve their basis vectors from the parent's arena, sized for the largest wave
  svar_handle* parent = nullptr;  // set on a view
  int view_w0 = 0;                // a view's first window in its parent
  std::map<std::pair<int, int>, svar_handle*> views;  // owned, by window range [w0, w1)
  double* arena = nullptr;
  int64_t arena_elems = 0;
  // Krylov workspace (grown on demand)
  int kry_gen = 0;  // bumped whenever the Krylov workspace below is (re)allocated
  struct Kry {
    int nrhs = -1, m = 0;
    int64_t ntot = 0;
    int64_t ldv = 0;  // element stride between basis vectors (ntot padded, see ensure_krylov)
    svar::KPlan plan;
    double *V = nullptr, *Z = nullptr, *u = nullptr, *w = nullptr, *z = nullptr;
    double *r = nullptr, *xs = nullptr, *part = nullptr, *npart = nullptr, *sums = nullptr;
    double* sysv = nullptr;
    double *tol_rel = nullptr, *hbuf = nullptr;
    svar::KState* st = nullptr;
    svar::KGlobal* gl = nullptr;
    svar::KHess* hs = nullptr;
    svar::KGlobal* gl_host = nullptr;  // pinned, two slots (lagged convergence checks)
    hipEvent_t gl_ev[2] = {nullptr, nullptr};
    int* net_off = nullptr;            // per system: learned correction switched off
    int* it0 = nullptr;                // per system: iterations of earlier cycles (history)
    int* flags = nullptr;              // operator skip flags: 1 + nsys + nwin (see Bases)
    // block (s-step) mode, allocated on first use: partial and reduced sums of the two
    // projections (stride slb per task / system), Gram partials and sums, per-system blocks
    double *bpart = nullptr, *bs1 = nullptr, *bs2 = nullptr, *gpart = nullptr, *gsum = nullptr;
    svar::KBlock* kb = nullptr;
    int slb = 0;
    // block FGMRES over the right-hand sides (allocated on first use): row tasks, per-window
    // states and Hessenberg storage, partial sums (stride br_slp per task), per-window sums
    // (stride br_sls): the two projections, the Gram matrices of the QR rounds, Y
    svar::KBRPlan br;
    svar::KBRWin* br_wins = nullptr;
    svar::KBRHess* br_hs = nullptr;
    double *br_part = nullptr, *br_c1 = nullptr, *br_c2 = nullptr, *br_g0 = nullptr;
    double *br_g1 = nullptr, *br_yl = nullptr, *br_hbuf = nullptr;
    int br_slp = 0, br_sls = 0;
    std::vector<void*> allocs;
  } kry;
};
