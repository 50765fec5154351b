/*
 * fracprec -- block-preconditioned FGMRES for the stabilized 3x3 block
 * Jacobian of frictional contact mechanics with hydraulically active
 * fractures, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Franceschini, Gazzola & Ferronato, "A scalable preconditioning
 * framework for stabilized contact mechanics with hydraulically active
 * fractures".  The system is the Newton system of Sec. 2.2 (eq. JacSys):
 *
 *     J = [ A   C1  Q1 ]   unknowns  u  (3 per mesh node, global frame)
 *         [ C2  -H  0  ]             t  (3 per fracture face, local frame)
 *         [ Q2  0   T  ]             p  (1 per fracture face)
 *
 * with the blocks of eq. block_def.  The preconditioner is M2 (t-u-p,
 * Alg 3.3 / 3.4, default) or M1 (t-p-u, Alg 3.1 / 3.2); the inner operator on
 * the mechanics Schur complement S1 = A + C1 H~^{-1} C2 (eq. Schur1_2) is one
 * smoothed-aggregation AMG V-cycle; the pressure block is solved exactly.
 *
 * Conventions for every entry point:
 *  - Vectors are device pointers (HIP global memory) of doubles, laid out
 *    [u (n_u) | t (n_t) | p (n_p)], u node-major (x, y, z per node), t
 *    face-major (N, T1, T2 per face), p in face order.  They are owned by the
 *    caller and must stay valid until the call returns.
 *  - All work is ordered on the HIP stream given to fpc_create; calls that
 *    return results to the host (fpc_info, convergence tests) synchronize
 *    that stream.
 *  - One handle per host thread.  A negative status means no output was
 *    written; fpc_last_error() returns a message.  FPC_NOT_CONVERGED (> 0) is
 *    a warning: the output holds the last iterate and the info its residual.
 *  - The library allocates device memory in fpc_setup (and once more on the
 *    first transposed call, for the transposed operators, and on the first
 *    single-column V-cycle of the t-u-p mode); fpc_apply_prec and fpc_solve
 *    allocate nothing after setup.
 */
#ifndef FRACPREC_H
#define FRACPREC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FPC_OK = 0,
  FPC_NOT_CONVERGED = 1,       /* warning: output holds the last iterate    */
  FPC_ERR_ARG = -1,            /* null pointer, bad option                   */
  FPC_ERR_DIM = -2,            /* block sizes inconsistent                   */
  FPC_ERR_PATTERN = -3,        /* CSR columns unsorted / duplicate / range   */
  FPC_ERR_SINGULAR_BLOCK = -4, /* a 3x3 face block of H or a coarse pivot    */
  FPC_ERR_NOT_SPD = -5,        /* nonpositive pivot of the pressure block    */
  FPC_ERR_NAN = -6,            /* NaN / Inf in values or right-hand side     */
  FPC_ERR_HIP = -7,            /* HIP runtime error                          */
  FPC_ERR_OOM = -8,            /* device allocation failed                   */
  FPC_ERR_STATE = -9,          /* call before fpc_setup                      */
  FPC_ERR_UNSUPPORTED = -10    /* case the library does not handle (message) */
} fpc_status;

enum { FPC_HOST = 0, FPC_DEVICE = 1 };
/* Preconditioner: t-u-p M2 (Alg 3.3 / 3.4), t-p-u M1 (Alg 3.1 / 3.2), or
 * M2* = D2^{-1} L2^{-1} of eq. LDU2 (the incomplete factorization of the
 * remark after Prop 3.2: one AMG call per application). */
enum { FPC_TUP = 0, FPC_TPU = 1, FPC_TUP_STAR = 2 };
enum { FPC_FP64 = 0, FPC_FP32_PREC = 1 };
/* Arnoldi orthogonalization of the single-right-hand-side FGMRES (the
 * paper does not fix it; Sec. 4 names GMRES only): classical Gram-Schmidt
 * applied twice (three passes over the basis per iteration), the textbook
 * modified Gram-Schmidt (j + 1 dependent dot products), or classical
 * Gram-Schmidt twice with the second projection delayed to the next step
 * (DCGS2 of Swirydowicz et al., Numer. Linear Algebra Appl. 2021: two passes
 * per iteration, the same Arnoldi relation in exact arithmetic; the last
 * column of a cycle takes one more pass). */
enum { FPC_CGS2 = 0, FPC_MGS = 1, FPC_DCGS2 = 2 };

/* Compressed sparse rows, 0-based, column indices strictly increasing in
 * every row.  Arrays live in host or device memory (fpc_block_system.ptr_space)
 * and are only read; fpc_setup deep-copies them. */
typedef struct {
  int64_t nrows, ncols, nnz;
  const int64_t* rowptr;   /* nrows + 1 */
  const int32_t* colind;   /* nnz */
  const double* val;       /* nnz */
} fpc_csr;

/* The seven blocks of eq. JacSys / eq. block_def.  Shapes: A n_u x n_u,
 * C1 n_u x n_t, Q1 n_u x n_p, C2 n_t x n_u, H n_t x n_t, Q2 n_p x n_u,
 * T n_p x n_p, with n_u = 3 * nodes and n_t = 3 * n_p.  Q2 may be empty.
 * coords: n_u/3 x 3 node coordinates (split node copies repeat theirs) for
 * the rigid-body near-nullspace, or NULL for translations only. */
typedef struct {
  int64_t n_u, n_t, n_p;
  fpc_csr A, C1, Q1, C2, H, Q2, T;
  const double* coords;
  int ptr_space;           /* FPC_HOST or FPC_DEVICE for every array above */
} fpc_block_system;

/* Smoothed-aggregation parameters (the paper leaves them open). */
typedef struct {
  int max_coarse;          /* coarsest level when dofs <= this (2000)      */
  int max_levels;          /* 12                                            */
  int cheb_degree;         /* Chebyshev degree, pre and post (2; only 2)    */
  double cheb_ratio;       /* interval [lambda_hi / ratio, lambda_hi] (5)   */
  int power_its;           /* power iterations for lambda (10)              */
  double lam_safety;       /* lambda_hi = safety * estimate (1.1)           */
  double omega_factor;     /* prolongator smoothing omega = f / lambda_hi   */
  double drop_tol;         /* dependent near-nullspace columns (1e-10)      */
} fpc_amg_options;

typedef struct {
  int mode;                /* FPC_TUP (default), FPC_TPU or FPC_TUP_STAR    */
  int precision;           /* FPC_FP64 or FPC_FP32_PREC (FP32 hierarchy)    */
  int restart;             /* FGMRES restart length (50; 1 to 63)           */
  int maxit;               /* total iteration cap (1000)                    */
  double rtol;             /* default relative tolerance (1e-8)             */
  int max_batch;           /* right-hand sides per fpc_solve_batch (32;   */
                           /* 1 to 32, larger values are rejected)          */
  int graphs;              /* 1: the batched V-cycle is captured once into  */
                           /* a HIP graph and replayed (default); 0: eager  */
  int ortho;               /* FPC_DCGS2 (default), FPC_CGS2 or FPC_MGS;     */
                           /* batched solves use DCGS2, or CGS2 for either  */
                           /* of the other two                              */
  int tune;                /* 0: each operator's apply layout follows from  */
                           /* its shape (default): two setups of one system */
                           /* give bitwise equal hierarchies,               */
                           /* preconditioners and solutions; 1: the         */
                           /* candidates are timed at setup and the fastest */
                           /* kept (the order of a product's sums may then  */
                           /* differ from setup to setup); 2: as 0, but     */
                           /* sliced ELL for rows of up to 32 blocks at any */
                           /* row count (small systems then take the layout */
                           /* of large ones)                                */
  fpc_amg_options amg;
} fpc_options;

typedef struct {
  int iterations;          /* FGMRES iterations (total over restarts)       */
  int restarts;            /* restart cycles                                */
  int converged;           /* 1 if the true residual met the tolerance      */
  double true_rel_residual;/* |b - J x| / |b| recomputed in FP64            */
  double est_rel_residual; /* last Givens estimate                          */
  double seconds;          /* wall time of the call                         */
} fpc_info;

/* Hierarchy description for one AMG level (tests and reporting). */
typedef struct {
  int64_t n_nodes;         /* block rows                                    */
  int64_t n_dofs;          /* real (unpadded) dofs                          */
  int block;               /* block size of the level (3 fine, 6 coarse)    */
  int64_t nnzb;            /* stored blocks of A_l                          */
  int64_t nnz_scalar;      /* nonzero scalar entries of A_l                 */
  int64_t p_nnzb, r_nnzb;  /* blocks of P_l and R_l = P_l^T                 */
  double lam_hi;           /* Chebyshev upper bound                         */
  int64_t n_agg;           /* aggregates formed on this level (0 coarsest)  */
  int layout[3];           /* apply layout picked for A_l, P_l, R_l: 1 =    */
                           /* sliced ELL, 4/16/64/256 = row groups of that  */
                           /* many lanes, 0 = none (coarsest)               */
  double tune_us[3];       /* with tune = 1, the winner's measured time per */
                           /* product (us); 0 when the rule picked it       */
} fpc_level_desc;

/* The pressure-block factorization (nested dissection, multifrontal; for
 * tests and reporting). */
typedef struct {
  int n_levels;            /* levels of the front tree (leaves = level 0)   */
  int64_t n_fronts;        /* fronts: leaves and non-empty separators        */
  int64_t factor_entries;  /* stored [F11^-1 | F11^-1 F12] entries, sum of   */
                           /* m (m + k) over fronts (m pivots, k boundary)  */
  int64_t solve_bytes;     /* algorithmic bytes of one single-column solve: */
                           /* factor read forward (m (m + k)) and backward  */
                           /* (m k) in FP64, plus vectors and index lists   */
  int64_t max_pivots;      /* largest m                                     */
  int64_t max_boundary;    /* largest k                                     */
} fpc_pressure_desc;

/* Fracture flow graph for the transmissibility gradient: TPFA face pairs
 * (K, L) (eq. FV_inner_product), Dirichlet edge counts and one-sided
 * transmissibilities.  Device pointers. */
typedef struct {
  int64_t n_p, n_pairs;
  const int32_t* pair_k;   /* n_pairs */
  const int32_t* pair_l;   /* n_pairs */
  const int32_t* ndir;     /* n_p */
  const double* upsilon;   /* n_p */
} fpc_flow_graph;

typedef struct fpc_handle fpc_handle;

/* Fill *opt with the defaults listed above (mode t-u-p, FP64, FGMRES(50),
 * rtol 1e-8, AMG: 2000 / 12 / degree 2 / ratio 5 / 10 its / 1.1 / 4/3 /
 * 1e-10). */
void fpc_default_options(fpc_options* opt);

/* Create a handle.  `stream` is a hipStream_t (NULL = default stream); the
 * handle does not own it.  *h is NULL on failure. */
fpc_status fpc_create(fpc_handle** h, const fpc_options* opt, void* stream);

/* Preconditioner construction, Alg 3.3 cpt_tup (or Alg 3.1 cpt_tpu):
 * H~ = Bdiag(H,3) and its inverse, S1 = A + C1 H~^{-1} C2 (eq. Schur1_2),
 * S~2 = T - FS(Q2, S1, Q1) (eq. FS_algebraic; zero when Q2 is empty) with
 * its exact inverse, and the smoothed-aggregation hierarchy of S1 with the
 * Galerkin products P^T A P.  Every array of *J is copied; the caller may
 * free them afterwards.  Open faces (a non-empty Q2, eq. Q2def) are handled
 * in every mode.  Errors: FPC_ERR_DIM / _PATTERN / _NAN on bad input,
 * FPC_ERR_SINGULAR_BLOCK for a singular face block of H, a singular pivot of
 * the pressure block or of the coarsest AMG level, FPC_ERR_NOT_SPD for a
 * nonpositive pivot of an SPD pressure block (Q2 empty, or t-p-u),
 * FPC_ERR_UNSUPPORTED when a face's fixed-stress index set K^(k) of
 * eq. Ak exceeds 64 scalar dofs, FPC_ERR_OOM.  A second call replaces the
 * previous setup. */
fpc_status fpc_setup(fpc_handle* h, const fpc_block_system* J);

/* Numeric re-setup for the next Newton or active-set iteration (Sec. 2.2:
 * the first block row does not change, C2, H and Q2 change in values and in
 * pattern as faces switch between stick, slip and open; Sec. 4: each
 * nonlinear iteration solves a new system with the same mesh).  Same sizes
 * as the setup; every block is uploaded and checked again and may have a new
 * pattern; the coordinates of the setup are kept.  When the block pattern of
 * the AMG operator (S1, or S~ in t-p-u with Q2 != 0) is unchanged, the
 * aggregates, tentative prolongators and apply layouts of the previous
 * hierarchy are reused (they depend on patterns and coordinates only) and
 * everything else is recomputed, so the result equals fpc_setup on the new
 * system; otherwise the hierarchy is rebuilt from scratch.  Likewise the
 * nested-dissection analysis of the pressure block is kept when its pattern
 * is unchanged, and its factor too when its values are bitwise unchanged
 * (with Q2 empty and the same T: always).  fpc_setup reuses nothing.  Errors as
 * fpc_setup; on error the handle is left not set up (FPC_ERR_STATE). */
fpc_status fpc_update_values(fpc_handle* h, const fpc_block_system* J);

/* 1 if the last fpc_setup / fpc_update_values reused the pattern-only parts
 * of the previous AMG hierarchy, 0 if it built them, -1 for a NULL handle. */
int fpc_hierarchy_reused(const fpc_handle* h);

/* v = M^{-1} w: Alg 3.4 app_tup (or Alg 3.2 app_tpu) with one V-cycle per
 * AMG(S1, .) call.  w, v: device, length n_u + n_t + n_p, distinct. */
fpc_status fpc_apply_prec(fpc_handle* h, const double* w, double* v);

/* v = M^{-T} w: the factors of eq. P2 (eq. P1) transposed in reverse order,
 * with the V-cycle on the transposed level operators. */
fpc_status fpc_apply_prec_T(fpc_handle* h, const double* w, double* v);

/* y = J x (trans = 0) or J^T x (trans = 1), eq. JacSys, FP64. */
fpc_status fpc_matvec(fpc_handle* h, int trans, const double* x, double* y);

/* One V-cycle x = AMG(S1, b) on the u block only (length n_u, device). */
fpc_status fpc_vcycle(fpc_handle* h, const double* b, double* x);

/* The pressure-block solve of the preconditioner by itself (device vectors
 * of length n_p): v = S~2^{-1} w (Alg 3.4 step 5; S~2 = T - FS(Q2, S1, Q1),
 * eq. app_Schur2_2, = T when Q2 = 0) in t-u-p and M2*, v = T^{-1} w (Alg 3.2
 * steps 1 and 7) in t-p-u; trans = 1 applies the transpose (the stored
 * inverse is symmetric, so the result is the same).  Runs on the handle's
 * stream, in FP64 with either precision of the hierarchy: forward and
 * backward sweeps over the levels of the nested-dissection factorization. */
fpc_status fpc_psolve(fpc_handle* h, int trans, const double* w, double* v);

/* Measurement aid, not a step of the method: a = b + scalar * c over n
 * doubles (device, 16-byte aligned), the STREAM triad used as the achievable
 * HBM bandwidth next to the roofline figures.  Any handle (set up or not)
 * supplies the stream. */
fpc_status fpc_stream_triad(fpc_handle* h, int64_t n, const double* b,
                            const double* c, double scalar, double* a);

/* Right-preconditioned FGMRES(restart) on J x = b (Sec. 4: zero initial
 * guess, stop at |b - J x| <= rtol |b|, the true residual recomputed in
 * FP64).  use_x0 != 0 starts from the values in x (restart / resume).
 * rtol <= 0 uses the handle's default.  info may be NULL. */
fpc_status fpc_solve(fpc_handle* h, const double* b, double* x, double rtol,
                     int use_x0, fpc_info* info);

/* Adjoint solve J^T lam = g with right preconditioner M^{-T}. */
fpc_status fpc_solve_T(fpc_handle* h, const double* g, double* lam,
                       double rtol, fpc_info* info);

/* k right-hand sides sharing J (k <= max_batch): column c of B is
 * B + c * ldb, of X is X + c * ldx (device, column-major).  Each column
 * runs its own FGMRES with its own tolerance rtol |b_c|; the preconditioner
 * is applied to all active columns at once.  infos: k entries or NULL. */
fpc_status fpc_solve_batch(fpc_handle* h, int k, const double* B, int64_t ldb,
                           double* X, int64_t ldx, double rtol,
                           fpc_info* infos);

/* dL/d(log Upsilon_K) = -lam_p^T (dT/d log Upsilon_K) p for a loss L(x)
 * whose adjoint pressure is lam_p (from fpc_solve_T): TPFA harmonic
 * averages and Dirichlet terms of eq. FV_inner_product.  lam_p, p, grad:
 * device, length n_p.  Every face pair is checked before use: an index
 * outside [0, n_p) or a pair (K, K) gives FPC_ERR_PATTERN and no output;
 * more than (2^31 - 2 n_p - 2) / 2 pairs give FPC_ERR_ARG.  Requires Q2 = 0
 * (FPC_ERR_UNSUPPORTED otherwise).  Each face sums its terms in ascending
 * pair order (deterministic).  Allocates a work area of 2 n_p + 1 + 2 n_pairs
 * int32 for the call. */
fpc_status fpc_grad_log_trans(fpc_handle* h, const fpc_flow_graph* g,
                              const double* lam_p, const double* p,
                              double* grad);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same result
 * as fpc_grad_log_trans, with the work area of 2 n_p + 1 + 2 n_pairs int32
 * taken from a static array of 2^20 int32 (4 MiB) that the library holds on
 * every device until the process ends; the call allocates and frees nothing.
 * A larger work area gives FPC_ERR_ARG and no output.  Every call on one GPU
 * shares that array (the parts that must start at zero are cleared by each
 * call): calls that overlap on one GPU, from several handles or threads,
 * race and must be serialized by the caller.  Errors as fpc_grad_log_trans. */
fpc_status fpc_grad_log_trans_noalloc(fpc_handle* h, const fpc_flow_graph* g,
                                      const double* lam_p, const double* p,
                                      double* grad);

/* The dense inverse of the coarsest AMG level (G17 of the smoothed-
 * aggregation setup: Gauss-Jordan with partial pivoting in 256-wide panels,
 * FP64 MFMA panel products) applied to a caller's matrix, for tests: D is a
 * device n x n row-major matrix (n <= 16384), replaced by its inverse.
 * FPC_ERR_SINGULAR_BLOCK (D unspecified) when a column has no nonzero pivot.
 * Any handle (set up or not) supplies the stream; allocates n^2 doubles
 * (n rounded up to a multiple of 64) for the call. */
fpc_status fpc_dense_inverse(fpc_handle* h, int64_t n, double* D);

/* Description of the pressure-block factorization (host output); zeros when
 * n_p = 0.  FPC_ERR_STATE before a successful setup. */
fpc_status fpc_pressure_info(const fpc_handle* h, fpc_pressure_desc* d);

/* Hierarchy introspection (host outputs). */
int fpc_num_levels(const fpc_handle* h);
fpc_status fpc_level_info(const fpc_handle* h, int level, fpc_level_desc* d);

/* Copy level data to host memory for checks: aggregate id per node (-1 =
 * isolated) of level `level` into agg (n_nodes int32); ranks (kept
 * near-nullspace columns per aggregate) into rank (n_agg int32).  Either
 * pointer may be NULL. */
fpc_status fpc_export_aggregates(const fpc_handle* h, int level, int32_t* agg,
                                 int32_t* rank);

/* Copy the BSR operator A_l (which = 0), P_l (1) or R_l (2) of a level to
 * host arrays: rowptr (nbrows+1), col (nnzb), val (nnzb * br * bc, blocks
 * row-major).  Query sizes with fpc_level_info. */
fpc_status fpc_export_level_matrix(const fpc_handle* h, int level, int which,
                                   int64_t* rowptr, int32_t* col, double* val);

/* Seconds spent in the phases of the last fpc_setup (host wall clock):
 * [0] total, [1] upload + validation, [2] H~ and S1, [3] pressure block,
 * [4] AMG hierarchy. */
fpc_status fpc_setup_times(const fpc_handle* h, double* t5);

/* Reporting aid: when enable != 0, the level-0 residual SpMV of every
 * V-cycle (the dominant kernel) is bracketed by HIP events on the handle's
 * stream.  Returns the number of timed launches and their total device time
 * (ms) accumulated since the last reset; reset != 0 clears the counters.
 * Synchronizes the stream. */
fpc_status fpc_kernel_timer(fpc_handle* h, int enable, int reset,
                            int64_t* launches, double* total_ms);

void fpc_destroy(fpc_handle* h);
const char* fpc_status_string(fpc_status s);
const char* fpc_last_error(const fpc_handle* h);

/* Counter-based hash used for aggregation priorities and power-iteration
 * start vectors (lowbias32, C. Wellons 2018), evaluated on the device for
 * n consecutive inputs starting at `first`; out: device, n uint32. */
fpc_status fpc_hash32_device(fpc_handle* h, uint32_t first, int64_t n,
                             uint32_t* out);

#ifdef __cplusplus
}
#endif

#endif /* FRACPREC_H */
