/*
 * svar.h -- C ABI of libsvar, an MI355X (gfx950) library for the preconditioned Krylov
 * solve of the linearised weak-constraint 4D-Var saddle-point system
 *
 *     [ D   0   L ] [d eta]   [ b ]
 *     [ 0   R   H ] [d nu ] = [ d ]        (Tabeart & Pearson, §2.1, eq. saddlepointsystem)
 *     [ L^T H^T 0 ] [d x  ]   [ 0 ]
 *
 * with D = blkdiag(B, Q_1..Q_N), R = blkdiag(R_0..R_N), H = blkdiag(H_0..H_N) and L block
 * lower-bidiagonal with identity diagonal and -M_i on the subdiagonal (eq. saddlepointA,
 * eq. def:L).  Time blocks are numbered i = 0..N; M_i maps the state at time i-1 to time i.
 *
 * Conventions for every call below.
 *  - Status: every function returns an int status (SVAR_OK on success).  On failure
 *    svar_last_error() returns a thread-local, NUL-terminated message that stays valid until
 *    the next call on the same thread.  No C++ exception crosses the ABI.
 *  - Descriptor arrays (svar_window_desc and what it points to) are HOST memory, float64 /
 *    int32, row-major; svar_create copies them to the device and the caller may free them
 *    on return.
 *  - Vector arguments of svar_apply_A / svar_apply_P / svar_apply_op / svar_solve are DEVICE
 *    pointers (float64) owned by the caller; the library never frees caller memory.  Input
 *    and output must not overlap.
 *  - Packed layout: windows in creation order; inside a window, nrhs vectors of that window
 *    one after another; a saddle vector of window w has length n_w = (2 s + pbar)(N+1) and
 *    holds (eta_0..eta_N | nu_0..nu_N | x_0..x_N), each eta_i / x_i of length s and nu_i of
 *    length p_i.  svar_offsets() returns the element offset of every window.
 *  - stream is a hipStream_t (NULL = default stream).  Calls are stream ordered and
 *    asynchronous except svar_create (synchronous set-up) and svar_solve, which synchronises
 *    the stream to read convergence flags and returns with info filled.  One handle must not
 *    be used from two streams or threads at once.
 */
#ifndef SVAR_H
#define SVAR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status codes */
#define SVAR_OK 0
#define SVAR_E_INVAL 1      /* bad argument or descriptor (message says which) */
#define SVAR_E_NOTSPD 2     /* a covariance (or Rhat / Dhat) is not symmetric positive definite */
#define SVAR_E_NOCONV 3     /* maxit reached; x holds the last iterate, info is filled */
#define SVAR_E_BREAKDOWN 4  /* non-finite value met in the Krylov recurrence */
#define SVAR_E_HIP 5        /* a HIP runtime call failed */
#define SVAR_E_NOMEM 6      /* device allocation failed */

/* ------------------------------------------------------------------ model maps M_i */
#define SVAR_MODEL_DENSE 0               /* M_i given as dense s x s matrices, i = 1..N       */
#define SVAR_MODEL_CIRC_BAND 1           /* (M x)_j = sum_t w_t x_{(j + off_t) mod s}, all i */
#define SVAR_MODEL_PERIODIC_TRIDIAG_INV 2/* M = T^{-1}, (T x)_j = a x_{j-1} + b x_j + c x_{j+1}
                                            periodic, same for all i (implicit advection-
                                            diffusion step)                                 */
#define SVAR_MODEL_L96_TLM 3             /* tangent linear of nsteps RK4 steps of Lorenz-96
                                            about a stored trajectory (see fields)          */
#define SVAR_MODEL_BAND_DIRICHLET 4      /* (M x)_j = sum_t w_t x_{j + off_t}, all i, with
                                            x_m = 0 outside 0..s-1 (homogeneous Dirichlet
                                            boundaries; e.g. the explicit heat-equation step
                                            of §7.2: offsets -1, 0, 1, weights r, 1 - 2r, r)  */

typedef struct svar_model_desc {
  int32_t kind;
  /* DENSE: dense[i-1] points to M_i (s x s, row-major), i = 1..N */
  const double* const* dense;
  /* CIRC_BAND (offsets taken modulo s) and BAND_DIRICHLET (|offsets| < s) */
  int32_t ntaps;
  const int32_t* offsets;   /* [ntaps] */
  const double* weights;    /* [ntaps] */
  /* PERIODIC_TRIDIAG_INV: a, b, c as above; |b| > |a| + |c| required */
  double tri_a, tri_b, tri_c;
  /* L96_TLM: dx_j/dt = (x_{j+1} - x_{j-2}) x_{j-1} - x_j + F (periodic, §7.1); M_i is the
     Jacobian of l96_nsteps RK4 steps of length l96_dt started from l96_traj[(i-1)*s ..]. */
  double l96_F, l96_dt;
  int32_t l96_nsteps;
  const double* l96_traj;   /* [N+1][s] linearisation states x_0..x_N (x_N unused) */
} svar_model_desc;

/* ------------------------------------------------------------------ one window */
typedef struct svar_window_desc {
  int32_t s;                 /* state size per time block                          */
  int32_t N;                 /* number of subwindows; blocks i = 0..N               */
  const int32_t* p;          /* [N+1] observations per block, p_i >= 0              */
  /* D_i = d_scale[i] * dmats[d_index[i]]  (B = D_0, Q_i = D_i)                    */
  int32_t n_dmat;
  const double* const* dmats;/* [n_dmat] s x s symmetric positive definite          */
  const int32_t* d_index;    /* [N+1]                                               */
  const double* d_scale;     /* [N+1] > 0                                           */
  /* R_i = rmats[r_index[i]], size p_i x p_i                                        */
  int32_t n_rmat;
  const double* const* rmats;/* [n_rmat] symmetric positive definite                */
  const int32_t* r_index;    /* [N+1]                                               */
  /* H_i in ELL form: row r of block i is sum_w h_vals[.][w] x_i[h_cols[.][w]]        */
  int32_t h_width;           /* entries per observation row, >= 1                   */
  const int32_t* h_cols;     /* [sum_i p_i * h_width], blocks concatenated, in [0,s) */
  const double* h_vals;      /* same shape                                          */
  svar_model_desc model;
} svar_window_desc;

/* ------------------------------------------------------------------ preconditioner options */
#define SVAR_PREC_NONE 0
#define SVAR_PREC_PD 1   /* block diagonal blkdiag(Dhat, Rhat, Lhat^T D^{-1} Lhat), eq. prec */
#define SVAR_PREC_PI 2   /* inexact constraint [[D,0,Lhat],[0,Rhat,0],[Lhat^T,0,0]], eq. prec */

#define SVAR_RHAT_DIAG 0   /* diag(R_i)                                          §5.1      */
#define SVAR_RHAT_RR 1     /* R_i + gamma I (ridge regression)                   Alg. 1    */
#define SVAR_RHAT_ME 2     /* eigenvalues below T raised to T (minimum eigenvalue) Alg. 2  */
#define SVAR_RHAT_EXACT 3  /* R_i itself                                                   */
#define SVAR_RHAT_BLOCK 4  /* R_block: R_i with the couplings between weakly correlated
                              groups of observation blocks removed              Alg. 3    */

typedef struct svar_prec_opts {
  int32_t type;      /* SVAR_PREC_*                                                        */
  int32_t k;         /* Lhat = L_M(k), 1 <= k <= N+1 (Definition 1; k = 1 gives L_0 = I)   */
  int32_t rhat;      /* SVAR_RHAT_*                                                        */
  double rr_gamma;   /* gamma of R_RR; < 0 selects lambda_min(R_i) (§6.1)                  */
  double me_T;       /* threshold of R_ME; < 0 selects the second smallest eigenvalue      */
  double d_ridge;    /* Dhat_i = D_i + d_ridge I (§6.1 uses 0.01); used by PD only         */
  /* R_block (Alg. 3, Appendix; rhat = SVAR_RHAT_BLOCK): R_i is split into rb_npvec blocks of
     sizes rb_pvec (host array, summing to p_i of every R matrix of the windows).  Where the
     scaled Frobenius norm ||R_i[block j, block j+1]||_F / sqrt(pvec_j pvec_{j+1}) of a
     super-diagonal block is below rb_tol, every coupling across that block boundary is
     removed; R_block keeps R_i whole inside each remaining group of blocks.  Then, once each:
     a group larger than rb_maxsize rows is split in two; with more groups than rb_numproc
     the two smallest adjacent groups are combined, with fewer than rb_numproc - 2 the
     largest group is split (a split cuts at the block boundary nearest the group's middle,
     a one-block group at its middle row; rb_maxsize, rb_numproc <= 0: no adjustment).
     Rhat^{-1} is then applied group by group. */
  const int32_t* rb_pvec;
  int32_t rb_npvec;
  int32_t rb_maxsize;
  double rb_tol;
  int32_t rb_numproc;
  int32_t lhat;      /* SVAR_LHAT_*: the approximation of L in both preconditioners          */
} svar_prec_opts;

#define SVAR_LHAT_LM 0   /* L_M(k) of Definition 1 (k above)                                  */
#define SVAR_LHAT_LI 1   /* L_I: every -M_i replaced by -I (§2.2); its inverse is the running
                            sum over the time blocks (k is not used)                          */

/* ------------------------------------------------------------------ solver options */
#define SVAR_METHOD_FGMRES 0  /* right-preconditioned flexible GMRES                    */
#define SVAR_METHOD_MINRES 1  /* preconditioned MINRES, needs SVAR_PREC_PD or NONE        */

#define SVAR_PRECISION_FP64 0         /* every operator in float64                       */
#define SVAR_PRECISION_MIXED_FP32 1   /* FP64 refinement; inner A float32, P float64     */
#define SVAR_PRECISION_MIXED_BF16P 2  /* FP64 refinement; inner A float32, P covariance
                                         products bfloat16 with float32 accumulation      */
#define SVAR_PRECISION_FP64_F32P 3    /* A in float64 (no refinement needed); P covariance
                                         products float32 (flexible GMRES absorbs them),
                                         except that FGMRES with P_I forms D z1 in float64
                                         (it is shared with the next A z)                  */
#define SVAR_PRECISION_FP64_BF16P 4   /* A in float64; P covariance products bfloat16 with
                                         float32 accumulation                              */
#define SVAR_PRECISION_MIXED_F32 5    /* FP64 refinement; every inner covariance product
                                         (A and P) float32 on the matrix cores with float32
                                         accumulation; FGMRES with P_I forms D z1 once in
                                         float32 and shares it with the next A z           */

typedef struct svar_solve_opts {
  int32_t method;     /* SVAR_METHOD_*                                                      */
  double rtol;        /* stop when ||rhs - A x||_2 <= rtol ||rhs||_2 (per right-hand side)  */
  int32_t maxit;      /* Krylov iterations allowed in total (per right-hand side)           */
  int32_t restart;    /* FGMRES basis size per cycle; 0 = no restart (one cycle of maxit)   */
  int32_t precision;  /* SVAR_PRECISION_*                                                   */
  double inner_rtol;  /* mixed precision: relative tolerance of each inner cycle            */
  int32_t max_outer;  /* refinement / restart cycles allowed (>= 1)                         */
  /* learned path (a network attached with svar_set_net): a FGMRES step fails when the
     least-squares residual does not fall below (1 - fallback_drop) times the previous one;
     after fallback_patience failing steps in a row the system's later preconditioner
     applications skip the network (the plain P).  With block_rhs the test runs per window on
     the two norm of its columns' residuals and switches the whole window.  fallback_drop <= 0
     disables the check. */
  double fallback_drop;
  /* training-pair harvest: when non-NULL, the state component v3 of the preconditioner input
     of each FGMRES step j < harvest_cap is copied to harvest + j * state_len (device memory,
     state_len = the packed state-space length of all windows and rhs).  Steps after every
     system has converged leave their slots untouched. */
  double* harvest;
  int32_t harvest_cap;
  int32_t fallback_patience;  /* >= 1 (values below 1 count as 1)                           */
  /* 1: replay FGMRES steps in chunks of 4 from a captured HIP graph (launched on a private
     stream ordered after / before the caller's stream with events); the results are those
     of the step-by-step launches.  Ignored while harvesting or timing. */
  int32_t use_graph;
  /* s-step FGMRES: block >= 2 builds the basis in blocks of `block` (at most 8) columns from
     one starting vector (preconditioner and A products back to back, each normalised), then
     orthogonalises the block against the basis with two block classical Gram-Schmidt passes
     and within itself with two Cholesky QR rounds: four reads of the basis per block instead
     of two per column.  With a linear preconditioner the iterates are those of one column at
     a time in exact arithmetic.  A block whose Gram matrix is numerically rank deficient is
     cut short and ends its cycle (the solve restarts from the float64 true residual while
     maxit allows).  Cycles hold at most 768 columns.  0 or 1: one column at a time.  A
     harvest then records every preconditioner input (the block's first vector and its
     normalised products); no graph replay in block mode. */
  int32_t block;
  /* MINRES stopping rule: 0 (default) the relative residual in the two norm, §7 -- the
     residual rhs - A x is carried along by the recurrence of A w (w the MINRES search
     directions, A w formed from the A v of each Lanczos step) and checked every iteration;
     1: the P^{-1}-norm estimate phibar <= rtol ||rhs||_{P^{-1}} of Paige-Saunders.  Either way
     the true residual is recomputed at return and a system whose ||rhs - A x||_2 exceeds
     rtol ||rhs||_2 reports SVAR_E_NOCONV.  Ignored by FGMRES. */
  int32_t minres_norm;
  /* residual history (nullable): DEVICE buffer of nsys * history_len doubles, nsys = windows x
     nrhs in packed order; entry [sys * history_len + t] receives the solver's residual-norm
     estimate (absolute, two norm; for MINRES with minres_norm = 1 the P^{-1}-norm estimate)
     after iteration t + 1, counting across restart and refinement cycles.  Entries after a
     system's last iteration are set to NaN.  Iterations beyond history_len are not recorded. */
  double* history;
  int32_t history_len;
  /* wave scheduling (FGMRES): the windows are solved in contiguous waves whose packed length
     (nrhs x the windows' saddle lengths) is at most wave_len elements, one wave after the
     other, so that the Krylov basis of a wave fits the device memory.  0: chosen from the
     free device memory (one wave when everything fits).  Each wave runs the same kernels on
     its windows; results equal those of one call up to the rounding order of the reductions.
     Not with harvest; MINRES always runs in one wave. */
  int64_t wave_len;
  /* block FGMRES over the right-hand sides (FGMRES, nrhs <= 8, block < 2, no harvest): 1 runs
     the nrhs systems of each window as one block -- the residuals are factorised R_0 = V_0 S_0,
     every step applies P and A to the nrhs columns of the newest basis block, orthogonalises
     the products against the basis (two block classical Gram-Schmidt passes) and within
     themselves (two Cholesky QR rounds), and the shared block Hessenberg matrix gives each
     column its own least-squares solution and residual estimate.  A window's cycle ends when
     every column meets its tolerance (its systems all stop together), when the basis is full,
     or when a new block loses rank (then the float64 restart continues).  Rank loss in the
     starting block (zero or equal residuals) puts seeded random directions in the basis.
     iters counts block steps (one P and one A product per system each).  Cycles hold at most
     7424 / nrhs^2 - 1 block steps (115 for 8 columns).  2: the same with one Gram-Schmidt
     pass per step (half the basis reads; the basis then loses orthogonality as classical
     Gram-Schmidt does, which restart cycles of a few tens of blocks keep near rounding).
     0: one Krylov space per system. */
  int32_t block_rhs;
} svar_solve_opts;

typedef struct svar_solve_info {   /* one per (window, right-hand side), packed order     */
  int32_t iters;        /* Krylov iterations used (all cycles)                              */
  int32_t outer;        /* refinement / restart cycles used                                 */
  int32_t status;       /* SVAR_OK, SVAR_E_NOCONV or SVAR_E_BREAKDOWN                       */
  int32_t fallbacks;    /* learned path: 1 if the network was switched off for this system  */
  double relres_true;   /* ||rhs - A x||_2 / ||rhs||_2 computed in float64 at return        */
  double relres_est;    /* the solver's own estimate at its last iteration                  */
  /* matrix-vector products with component blocks, counted as in Tables 4 and 5 but as
     formed: under P_I with a float64 operator, FGMRES forms D z1 once per step (inside P)
     and the next A z reuses it, so n_D counts one D product per step there */
  int64_t n_M, n_MT, n_D, n_R, n_Rhat_inv, n_Dhat_inv;
} svar_solve_info;

typedef struct svar_handle svar_handle;

/* Create a handle for nwin windows (all with the same preconditioner options).  Copies the
   descriptors to the device of the calling thread, then builds Rhat^{-1} and Dhat^{-1} on
   the GPU (§6.2: Rhat_i is precomputed before the iteration).  Synchronous. */
int svar_create(const svar_window_desc* windows, int32_t nwin, const svar_prec_opts* popts,
                svar_handle** out, void* stream);

/* Release every device buffer of the handle.  NULL is accepted. */
int svar_destroy(svar_handle* h);

/* Per-RHS saddle vector length n_w of window w (or -1 if w is out of range). */
int64_t svar_system_size(const svar_handle* h, int32_t w);

/* off[w] = element offset of window w in a packed vector of nrhs right-hand sides per window;
   off[nwin] = total length.  off must hold nwin + 1 entries (host memory). */
int svar_offsets(const svar_handle* h, int32_t nrhs, int64_t* off);

/* y = A v for every window and right-hand side (§6.2: c1 = D v1 + L v3, c2 = R v2 + H v3,
   c3 = L^T v1 + H^T v2). */
int svar_apply_A(svar_handle* h, int32_t nrhs, const double* v, double* y, void* stream);

/* z = P^{-1} v with the handle's preconditioner (§6.2):
   P_D^{-1} v = (Dhat^{-1} v1, Rhat^{-1} v2, Lhat^{-1} D Lhat^{-T} v3),
   P_I^{-1} v = (c1 = Lhat^{-T} v3, Rhat^{-1} v2, Lhat^{-1}(v1 - D c1)). */
int svar_apply_P(svar_handle* h, int32_t nrhs, const double* v, double* z, void* stream);

/* The operators of the inner loop of the mixed-precision solves (§6.2 maps with reduced-
   precision covariance products, float32 accumulation).  precision = SVAR_PRECISION_FP64 is
   svar_apply_A / svar_apply_P; for A both MIXED settings use float32 copies of D and R
   (FP64_F32P keeps A in float64); for P, SVAR_PRECISION_MIXED_BF16P uses bfloat16 copies of D,
   Rhat^{-1} and Dhat^{-1}, SVAR_PRECISION_FP64_F32P float32 copies, and
   SVAR_PRECISION_MIXED_FP32 the float64 preconditioner.  Vectors stay float64. */
int svar_apply_A_prec(svar_handle* h, int32_t precision, int32_t nrhs, const double* v, double* y,
                      void* stream);
int svar_apply_P_prec(svar_handle* h, int32_t precision, int32_t nrhs, const double* v, double* z,
                      void* stream);

/* y = A v like svar_apply_A, for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, harnesses that forbid allocation): it allocates nothing
   and builds nothing.  The launch program of this nrhs must already exist (an earlier
   svar_apply_A call with the same handle and nrhs builds it; otherwise SVAR_E_INVAL).  The
   split-K partial sums of the covariance products go to a static device array of the library
   (8 Mi doubles = 64 MiB per GPU, held until the process ends) instead of the handle's
   workspace; a program that needs more returns SVAR_E_INVAL.  Every call on one GPU shares
   that array: calls that overlap on one GPU (several streams or threads) race.  Results are
   bitwise those of svar_apply_A; no kernel-class timing is recorded. */
int svar_apply_A_noalloc(svar_handle* h, int32_t nrhs, const double* v, double* y, void* stream);

/* Component maps, for checking each step on its own.  Vectors of the "state" space hold
   (N+1) s entries per (window, rhs); those of the "obs" space hold sum_i p_i entries; packed
   window by window and rhs by rhs like saddle vectors. */
#define SVAR_OP_L 0           /* state -> state: L x                                    */
#define SVAR_OP_LT 1          /* state -> state: L^T x                                  */
#define SVAR_OP_LHAT_INV 2    /* state -> state: L_M(k)^{-1} x                          */
#define SVAR_OP_LHAT_INVT 3   /* state -> state: L_M(k)^{-T} x                          */
#define SVAR_OP_D 4           /* state -> state: D x                                    */
#define SVAR_OP_DHAT_INV 5    /* state -> state: Dhat^{-1} x (needs a PD handle)        */
#define SVAR_OP_R 6           /* obs -> obs: R y                                        */
#define SVAR_OP_RHAT_INV 7    /* obs -> obs: Rhat^{-1} y                                */
#define SVAR_OP_H 8           /* state -> obs: H x                                      */
#define SVAR_OP_HT 9          /* obs -> state: H^T y                                    */
int svar_apply_op(svar_handle* h, int32_t op, int32_t nrhs, const double* in, double* out,
                  void* stream);

/* Solve A x = rhs for nrhs right-hand sides per window, x0 = 0.  info: host array of
   nwin * nrhs entries (packed order).  Returns SVAR_OK when every system met rtol,
   SVAR_E_NOCONV / SVAR_E_BREAKDOWN when one did not (x then holds its last iterate). */
int svar_solve(svar_handle* h, const svar_solve_opts* opts, int32_t nrhs, const double* rhs,
               double* x, svar_solve_info* info, void* stream);

/* Outer (Gauss-Newton) loop support, §2.1: the increments b_i = M_i(x_{i-1}) - x_i need the
   model itself.  y_0 = x_0 and y_i = M_i(x_{i-1}) for i = 1..N, one observation interval of the
   model of window w (nonlinear for SVAR_MODEL_L96_TLM: l96_nsteps RK4 steps; the linear map for
   the other kinds).  x, y: device state vectors of (N+1) s doubles, distinct buffers. */
int svar_model_forecast(svar_handle* h, int32_t w, const double* x, double* y, void* stream);

/* Replace the linearisation states x_0..x_N of a Lorenz-96 window (device pointer, (N+1) s
   doubles, copied), e.g. after an outer-loop update.  E_INVAL for other model kinds. */
int svar_set_trajectory(svar_handle* h, int32_t w, const double* traj, void* stream);

/* Right-hand side of the outer loop's saddle system (§2.1, incremental form) for window w of
   a handle whose right-hand sides hold one system (nrhs = 1 layout of that window): with the
   current trajectory x = (x_0..x_N), the background x_b and the observations y,
       b_0 = x_b - x_0,  b_i = M_i(x_{i-1}) - x_i (i = 1..N),  d_i = y_i - H_i x_i,
   and the third component zero.  x: device state vector ((N+1) s), xb: device (s), y: device
   observation vector (sum_i p_i, blocks concatenated), rhs: device saddle vector of the
   window (n_w doubles), distinct from the inputs.  Stream ordered. */
int svar_gn_rhs(svar_handle* h, int32_t w, const double* x, const double* xb, const double* y,
                double* rhs, void* stream);
/* Outer-loop update x += dx with dx the state component of the saddle solution sol (device,
   n_w doubles); for Lorenz-96 windows also the new linearisation trajectory of the window
   (svar_set_trajectory), so the next solve uses the tangent linear model about x. */
int svar_gn_update(svar_handle* h, int32_t w, double* x, const double* sol, void* stream);

/* Set-up results of window w: gamma of R_RR, T of R_ME and lambda_1(R_i) for each distinct
   R matrix (host arrays of n_rmat entries; NaN where not applicable; any may be NULL). */
int svar_rhat_params(const svar_handle* h, int32_t w, double* gamma, double* T, double* lam1);

/* Kernel timing: when enabled, the library records HIP events around every launch of the
   given kernel class on the caller's stream and accumulates their durations. */
#define SVAR_KCLASS_GEMM 0      /* covariance products (D, R, Rhat^{-1}, Dhat^{-1})      */
#define SVAR_KCLASS_ORTHO 1     /* Gram-Schmidt passes of FGMRES                          */
#define SVAR_KCLASS_MODEL 2     /* model products and Lhat sweeps                         */
#define SVAR_KCLASS_NET 3       /* learned correction (sigma, network inference, update)  */
#define SVAR_KCLASS_COUNT 4
int svar_timing_enable(svar_handle* h, int32_t kclass, int32_t on);
/* total_ms, launches: host pointers; resets the accumulators when reset != 0. */
int svar_timing_read(svar_handle* h, int32_t kclass, double* total_ms, int64_t* launches,
                     int32_t reset);

/* ------------------------------------------------------------------ learned correction
   Both preconditioners apply Lhat^{-T} = L_M(k)^{-T} (Definition 1) to v3: P_I as its first
   output c1 (which also feeds the Schur term Lhat^{-1} D c1), P_D inside its Schur-complement
   approximation Lhat^{-1} D Lhat^{-T} v3 (§2.2, §6.2).  With P(i, j) = M_{i+1}^T ... M_j^T the
   exact sweep differs from the truncated one at block i by sum_m P(i, b_m) chat_{b_m} over the
   later segment starts b_m = e(i) + 1 + (m - 1) k, where e(i) ends block i's segment.  A
   network corrects the sweep output towards the exact L^{-T} v3:
       c = chat + sigma * NN(features(chat / sigma)),   sigma = rms of chat over the system,
   features of block i: chat_i, chat at the next n_bound segment starts (zero past block N),
   one-hot of e(i) - i.  NN: periodic 1D convolutions over space of width 5,
   (1 + n_bound + k) -> 64 -> 64 -> 64 -> 1 channels, ReLU after the first three.
   Parameters (float32, host order): W1 (64, cin, 5), b1 (64), W2 (64, 64, 5), b2, W3, b3,
   W4 (1, 64, 5), b4 (1), each row-major.  Training: mean squared error, Adam. */
#define SVAR_NET_FP32 0   /* inference with float32 MFMA                                 */
#define SVAR_NET_BF16 1   /* inference with bfloat16 weights and activations, float32
                             accumulation                                                 */

typedef struct svar_net svar_net;
typedef struct svar_net_desc {
  int32_t k;          /* segment length of the corrected sweep (the handle's k), >= 1      */
  int32_t n_bound;    /* later segment starts used as inputs, >= 0, 1 + n_bound + k <= 32  */
  int32_t precision;  /* SVAR_NET_* of the inference inside the preconditioner             */
  int32_t pad;
} svar_net_desc;
typedef struct svar_adam_opts {
  double lr, beta1, beta2, eps;  /* Adam (Kingma & Ba) with bias correction               */
} svar_adam_opts;

/* Create a network on the calling thread's device with zero parameters. */
int svar_net_create(const svar_net_desc* desc, svar_net** out);
/* Release it (NULL accepted).  A handle it is attached to must be detached first. */
int svar_net_destroy(svar_net* net);
/* Number of float32 parameters, or -1 for NULL. */
int64_t svar_net_nparams(const svar_net* net);
/* Copy all parameters from / to host memory (nparams floats); set_params also clears the
   Adam state.  Synchronous. */
int svar_net_set_params(svar_net* net, const float* theta);
int svar_net_get_params(const svar_net* net, float* theta);

/* Training pairs of npair systems of nb blocks of s points (device memory): chat is the
   truncated sweep output, cexact the exact one (both float64, [npair][nb][s]); writes
   x = chat / sigma and y = (cexact - chat) / sigma as float32 (zeros where sigma = 0). */
int svar_net_make_pairs(int32_t npair, int32_t nb, int32_t s, const double* chat,
                        const double* cexact, float* x, float* y, void* stream);

/* out[p][i][j] = NN(features(x_p))[i][j] for normalised sweep outputs x ([npair][nb][s]
   float32, device); precision SVAR_NET_*. */
int svar_net_forward(svar_net* net, int32_t precision, int32_t npair, int32_t nb, int32_t s,
                     const float* x, float* out, void* stream);

/* One float32 training step on the blocks samples[2 q] (pair) / samples[2 q + 1] (block),
   q < nsample (host array) of the pairs (x, y) ([npair][nb][s] float32, device): the loss
   sum over those blocks of (NN - y)^2 / (nsample s), its gradient, and, when adam is not
   NULL, one Adam update.  loss (host double) and grad (host, nparams floats, the gradient
   before the update) may be NULL; asking for either synchronises the stream. */
int svar_net_train_step(svar_net* net, int32_t npair, int32_t nb, int32_t s, const float* x,
                        const float* y, int32_t nsample, const int32_t* samples,
                        const svar_adam_opts* adam, double* loss, float* grad, void* stream);

/* Training loop on a pair pool: `epochs` passes over every (pair, block) sample of (x, y)
   ([npair][nb][s] float32, device, as written by svar_net_make_pairs), in mini-batches of
   `batch` samples, each a float32 forward / backward pass and one Adam step
   (svar_net_train_step).  The sample order of epoch e is a Fisher-Yates shuffle driven by
   splitmix64 seeded with seed + e.  When ckpt_path is not NULL a checkpoint (parameters,
   Adam moments and step count, and the data cursor: the epoch and the position of the next
   batch in that epoch's order) is written after every checkpoint_every Adam steps (0: none
   inside an epoch) and at the end of every epoch, to ckpt_path + ".tmp" and then renamed.
   resume = 1 continues from the checkpoint at ckpt_path when the file exists (it must
   belong to the same pool shape, seed and batch size): the continued run reproduces the
   uninterrupted one.  loss_hist (host, epochs doubles, nullable): mean loss of each epoch
   (asking for it synchronises after every step).  Synchronous. */
typedef struct svar_train_opts {
  int32_t epochs;
  int32_t batch;
  svar_adam_opts adam;
  uint64_t seed;
  int32_t checkpoint_every;
  int32_t resume;
} svar_train_opts;
int svar_train(svar_net* net, int32_t npair, int32_t nb, int32_t s, const float* x,
               const float* y, const svar_train_opts* opts, const char* ckpt_path,
               double* loss_hist, void* stream);
/* Load a checkpoint written by svar_train into a network of the same k, n_bound and size:
   parameters and Adam state.  cursor (host, 3 int64, nullable) receives the epoch, the
   position in that epoch's order and the Adam step count.  Synchronous. */
int svar_load_learned(svar_net* net, const char* path, int64_t* cursor);

/* Attach (or with NULL detach) a network to a handle: svar_apply_P and svar_solve then
   correct every Lhat^{-T} v3 of the preconditioner as above.  The network's k must equal
   the handle's; it must outlive the attachment.  Training it later changes the correction. */
int svar_set_net(svar_handle* h, svar_net* net);

/* Tile autotuning of the covariance products (matrix-panel GEMMs): for every GEMM launch of
   the A and P programs of nrhs right-hand sides at `precision` (SVAR_PRECISION_*), time the
   candidate plans (k-split kernel or LDS-tiled kernel, several workgroup counts; one warm-up
   and five timed launches on zero-filled scratch vectors, HIP events on `stream`), keep the
   fastest per shape key (precision | n x ncols of each product) in the handle and rebuild the
   programs with it.  Shapes already tuned are skipped.  When cache_path is not NULL the
   choices are merged into that JSON file (one entry per line: key, tiled, target, us,
   default_us).  Synchronous.  Results do not depend on the plan beyond rounding order. */
int svar_autotune(svar_handle* h, int32_t nrhs, int32_t precision, const char* cache_path,
                  void* stream);
/* Load the choices of a cache written by svar_autotune (unknown shapes keep the default). */
int svar_autotune_load(svar_handle* h, const char* cache_path);

/* Spectral diagnostics (Theorem 1, Propositions 1-4): nsteps steps of the Lanczos process for
   the eigenvalues of M^{-1} K on window w, in the M inner product, from the caller's start
   vector (device, the operator's space of window w, length: SPEC_PD_A n_w, SPEC_RHAT_R
   sum_i p_i, SPEC_LML (N+1) s).  ritz (host, nsteps doubles) receives the eigenvalues of the
   Lanczos tridiagonal in ascending order and *nritz their number (fewer than nsteps when the
   Krylov space becomes invariant).  The extreme Ritz values approach the extreme eigenvalues
   first; without re-orthogonalisation converged values can repeat.  Synchronous. */
#define SVAR_SPEC_PD_A 0    /* P_D^{-1} A, K = A, M = P_D (needs a P_D handle)                  */
#define SVAR_SPEC_RHAT_R 1  /* Rhat^{-1} R over all observation blocks, K = R, M = Rhat       */
#define SVAR_SPEC_LML 2     /* Lhat^{-T} L^T L Lhat^{-1} (Lhat = L_M(k) or L_I), M = I          */
int svar_spectrum(svar_handle* h, int32_t which, int32_t w, int32_t nsteps, const double* start,
                  double* ritz, int32_t* nritz, void* stream);

const char* svar_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SVAR_H */
