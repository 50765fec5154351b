// Apply-path entry points (V-cycle, block-preconditioner pieces, Krylov).
#pragma once

#include "fpc_handle.hpp"

namespace fpc {

template <typename T>
CycleVecs<T>& cycle_vecs(Hierarchy& H, int nv);
// One V-cycle on NV interleaved columns: input cycle_vecs(H,NV).lv[0].b,
// output .lv[0].xo.
template <typename T, int NV>
void vcycle(Hierarchy& H, bool transpose, hipStream_t s);
// Single-column cycle whose input is formed by vcycle_input (as to_level on
// the finest level's b, plus that level's first Chebyshev direction when the
// coupling blocks have row lists: the return value) and whose result goes,
// in FP64, straight to out from the last smoothing product.
template <typename T>
bool vcycle_input(Hierarchy& H, const double* base, const Csr* m1,
                  const double* x1, double a1, const Csr* m2,
                  const double* x2, double a2, hipStream_t s);
template <typename T>
void vcycle_to(Hierarchy& H, bool transpose, bool d0_ready, double* out,
               hipStream_t s);

// Apply layout of one operator picked by timing the candidates with `nv`
// columns (option tune = 1); *choice = 1 for
// sliced ELL, else the row-group width.
// `sell`: the operator's sliced-ELL layout if already built (taken over).
template <typename T>
void tune_op(const Bsr& M, int nv, Op<T>& out, hipStream_t s, int* choice,
             double* best_us, Sell<T>* sell = nullptr);

// The apply layout chosen from the shape alone (no timing, so the same for
// every setup of a pattern): rows of more than 32 blocks take row groups of
// 16 lanes below 64 blocks per row and of 64 lanes above (a workgroup of 256
// lanes for fewer than 4,096 rows of 256 blocks or more); shorter rows take
// sliced ELL when there are at least 65,536 of them (1,024 slices, enough to
// fill the GPU with one lane per row) or when any_rows is set, row groups of
// 16 or 4 lanes (from 16 blocks per row) otherwise.
int rule_layout(const Bsr& M, bool any_rows = false);

// The apply layout `choice` (as returned by tune_op) of one operator.
template <typename T>
void build_op(const Bsr& M, int choice, Op<T>& out, hipStream_t s,
              Sell<T>* sell = nullptr);

void sell_mv(const Sell<double>& A, const double* x, double* y, hipStream_t s);
void sell_mv_dinv(const Sell<double>& A, const double* dinv, const double* x,
                  double* y, hipStream_t s);
void face_apply(const double* hinv, const double* in, double* out,
                int64_t n_p, int trans, hipStream_t s);
template <typename T>
void to_level(T* out, int nv, int colv, int64_t n, const double* base,
              const Csr* m1, const double* x1, double a1, const Csr* m2,
              const double* x2, double a2, hipStream_t s);
template <typename T>
void from_level(const T* xo, int nv, int64_t n, double* vu, int diff,
                hipStream_t s);
void tface(const Csr& C, const double* vu, const double* t_t,
           const double* hinv, double* v_t, int64_t n_p, int trans,
           hipStream_t s);
// ---------------------------------------------------------------- k_pnd
// Ordering (nested dissection) and symbolic analysis of the pressure block's
// pattern; flags[FLAG_PATTERN] for an unsymmetric matrix,
// flags[FLAG_OVERFLOW] for a front boundary beyond 4096 faces.
void psolve_analyse(PSolve& ps, const Csr& T, int* flags, hipStream_t s);
// Numeric factorization of T - diag(sk) (sk nullable) on the analysis.
void psolve_factor(PSolve& ps, const Csr& T, const double* sk, bool spd,
                   int* flags, hipStream_t s);
int64_t psolve_factor_entries(const PSolve& ps);
// Algorithmic bytes of one single-column solve: factor entries read by the
// forward (m (m + k)) and backward (m k) sweeps, FP64; input gathered and
// output scattered through perm (8 + 4 bytes per face each); c_S written and
// read back (16 per face); contributions written and gathered (16 + 4 per
// slot); boundary indices of the backward sweep (4 per slot).
int64_t psolve_solve_bytes(const PSolve& ps);
void psolve_apply(const PSolve& ps, const double* in, double* out,
                  int64_t n_p, int trans, hipStream_t s);
void psolve_batch_buffers(PSolve& ps, int KB);

// ---------------------------------------------------------------- batches
void sell_mv_b(const Sell<double>& A, const double* x, double* y, int KB,
               hipStream_t s);
void pack_cols(const double* B, int64_t ldb, int64_t n, int k, int KB,
               double* out, hipStream_t s);
void unpack_cols(const double* Xi, int64_t n, int k, int KB, double* X,
                 int64_t ldx, hipStream_t s);
void face_apply_b(const double* hinv, const double* in, double* out,
                  int64_t n_p, int KB, int trans, hipStream_t s);
void csr_spmv2_b(const Csr* m1, const double* x1, double a1, const Csr* m2,
                 const double* x2, double a2, double* y, double beta, int KB,
                 hipStream_t s);
template <typename T>
void to_level_b(T* out, int KB, int64_t n, const double* base,
                const Csr& M1, const double* x1, double a1, const Csr& M2,
                const double* x2, double a2, hipStream_t s);
template <typename T>
void from_level_b(const T* xo, int64_t n, int KB, double* vu, hipStream_t s);
void tface_b(const Csr& C, const double* vu, const double* t_t,
             const double* hinv, double* v_t, int64_t n_p, int KB,
             hipStream_t s);
void psolve_apply_b(const PSolve& ps, const double* in, double* out,
                    int64_t n_p, int KB, hipStream_t s);
void bmdot(const double* V, int64_t ldv, int nv, const double* W, int64_t n,
           int KB, double* part, double* out, hipStream_t s);
// Batched Gram-Schmidt passes (as cgs_dot / cgs_axpy_dot / cgs_axpy_norm,
// per column; out[o * KB + c]); partials sized by bdot_partials.
int64_t bdot_partials(int nv, int KB);
void bcgs_dot(const double* V, int64_t ldv, int nv, const double* W, int64_t n,
              int KB, double* part, double* out, hipStream_t s);
void bcgs_axpy_dot(const double* V, int64_t ldv, int nv, const double* h,
                   double* W, int64_t n, int KB, double* part, double* out,
                   hipStream_t s);
void bcgs_axpy_norm(const double* V, int64_t ldv, int nv, const double* h,
                    double* W, int64_t n, int KB, double* part, double* out,
                    hipStream_t s);
void bmaxpy(const double* V, int64_t ldv, int nv, const double* h, double* W,
            int64_t n, int KB, hipStream_t s);
void bscale(const double* x, const double* scal, double* y, int64_t n, int KB,
            hipStream_t s);
void bsub(const double* a, double* b, int64_t n, hipStream_t s);
void bgmres_step(double* H, double* cs, double* sn, double* g,
                 const double* h1, const double* h2, const double* nrm2,
                 const double* nrm0, int j, int m, int KB, const int* active,
                 double* scal, double* est, int* brk, hipStream_t s);
// Batched delayed Gram-Schmidt (the dcgs_* steps per column of the
// interleaved block; D and P hold column c of output o at [o * KB + c], sc
// holds the provisional estimates [0, KB), the final ones [KB, 2 KB) and
// the step codes [2 KB, 3 KB) as doubles).
bool bdcgs_supported(int64_t n, int KB);
void bdcgs_dot(const double* V, int64_t ldv, int nv, const double* U,
               const double* W, int64_t n, int KB, double* part, double* D,
               hipStream_t s);
void bdcgs_finish(const double* D, int nv, bool fresh, const int* needfin,
                  double* H, int m, double* cs, double* sn, double* g,
                  double* P, double* rho, double* ww, double* sc, int* pf,
                  const int* active, int KB, hipStream_t s);
void bdcgs_update(double* V, int64_t ldv, int j, const double* D,
                  const double* P, const double* rho, const double* W,
                  int64_t n, int KB, double* part, hipStream_t s);
void bdcgs_peek(const double* part, int64_t n, double* H, int m, double* cs,
                double* sn, double* g, const double* P, int j,
                const double* ww, double* sc, int* pf, const int* active,
                int KB, hipStream_t s);
void bgmres_init(double* g, int m, int KB, const double* beta2,
                 const int* active, double* scal, hipStream_t s);
void btrisolve(const double* H, const double* g, double* y, const int* kc,
               int m, int KB, hipStream_t s);

// ---------------------------------------------------------------- Krylov
// partial[i * G + blk] = <V_i, w> over a chunk; V_i = V + i * ldv
constexpr int kDotBlocks = 256;
// Size of the partials buffer mdot needs for nv vectors of length n.
int64_t mdot_partials(int64_t n, int nv);
void mdot(const double* V, int64_t ldv, int nv, const double* w, int64_t n,
          double* partials, double* out, hipStream_t s);
// Classical Gram-Schmidt passes (partials sized by mdot_partials):
//   cgs_dot:       out[i] = <V_i, w> (i < nv), out[nv] = <w, w>
//   cgs_axpy_dot:  w -= sum_i h_i V_i, then out[i] = <V_i, w>
//   cgs_axpy_norm: w -= sum_i h_i V_i, then out[0] = <w, w>
void cgs_dot(const double* V, int64_t ldv, int nv, const double* w, int64_t n,
             double* partials, double* out, hipStream_t s);
void cgs_axpy_dot(const double* V, int64_t ldv, int nv, const double* h,
                  double* w, int64_t n, double* partials, double* out,
                  hipStream_t s);
void cgs_axpy_norm(const double* V, int64_t ldv, int nv, const double* h,
                   double* w, int64_t n, double* partials, double* out,
                   hipStream_t s);
// Gram-Schmidt twice with the second projection delayed by one step
// (partials sized by mdot_partials for 2 kMaxKrylov + 1 vectors).  Slot j
// of V holds u_j (unnormalized remainder of step j-1), V_0 .. V_{j-1} are
// final.
//   dcgs_dot:    D[i] = <V_i, u>, and with w: D[nv + i] = <V_i, w>,
//                D[2 nv] = <w, w> (i < nv; the last vector may be u itself)
//   dcgs_finish: rho_j into scal[0]; fin: column j-1 of H final (P + a,
//                subdiagonal rho_j) and committed, estimate in scal[5],
//                ctrl[0] = 2 if rho_j = 0; fresh: first projection of
//                column j into P, <w, w> into scal[6]
//   dcgs_update: slot j <- v_j, slot j+1 <- u_{j+1}, partials of |u_{j+1}|^2
//   dcgs_peek:   provisional estimate of column j into scal[1]; on
//                breakdown the column is committed, scal[5] set, ctrl[0] = 1
// (dcgs_finish and dcgs_peek also leave ctrl[0] in scal[7], as a double, so
// that one copy of scal brings every scalar the host tests)
bool dcgs_supported(int64_t n);
void dcgs_dot(const double* V, int64_t ldv, int nv, const double* u,
              const double* w, int64_t n, double* partials, double* D,
              hipStream_t s);
void dcgs_finish(const double* D, int nv, bool fin, bool fresh, double* H,
                 int ldh, double* cs, double* sn, double* g, double* P,
                 double* scal, int* ctrl, hipStream_t s);
void dcgs_update(double* V, int64_t ldv, int j, const double* D,
                 const double* P, const double* scal, const double* w,
                 int64_t n, double* partials, hipStream_t s);
void dcgs_peek(const double* partials, int64_t n, double* H, int ldh,
               double* cs, double* sn, double* g, const double* P, int j,
               double* scal, int* ctrl, hipStream_t s);
// w -= sum_i h_i V_i
void maxpy(const double* V, int64_t ldv, int nv, const double* h, double* w,
           int64_t n, hipStream_t s);
// y = x * (1 / scal[0]) (scal on device); if scal[0] == 0 y = 0
void scale_by_inv(const double* x, const double* scal, double* y, int64_t n,
                  hipStream_t s);
// y = a * x + b * y
void axpby(double a, const double* x, double b, double* y, int64_t n,
           hipStream_t s);
// FGMRES step j on device: H[:, j] = h1 + h2 (j+1 entries), H[j+1, j] =
// sqrt(nrm2); Givens update of H, cs, sn, g; scal[0] = H[j+1,j] before
// rotation (0 on breakdown), scal[1] = |g_{j+1}|, ctrl[0] = scal[7] =
// breakdown.
void gmres_step(double* H, int ldh, double* cs, double* sn, double* g,
                const double* h1, const double* h2, const double* nrm2,
                const double* nrm2_before, int j, double* scal, int* ctrl,
                hipStream_t s);
void gmres_init(double* g, int m, const double* beta2, double* scal,
                hipStream_t s);
// y = R^{-1} g, R = H[0:k, 0:k] upper triangular
void gmres_trisolve(const double* H, int ldh, const double* g, double* y,
                    int k, hipStream_t s);
void sqrt_dev(const double* in, double* out, hipStream_t s);

// ---------------------------------------------------------------- device
// Base of vector i (clamped to nv - 1) as a wavefront-uniform pointer, so
// that a load takes it from scalar registers with a 32-bit per-lane offset.
typedef const __attribute__((address_space(1))) char* gchar_ptr;

__device__ inline gchar_ptr cgs_base(const double* V, uint64_t stride_b, int i,
                                     int nv) {
  const int ie = i < nv ? i : nv - 1;
  const uint64_t a = reinterpret_cast<uint64_t>(V) + (uint64_t)ie * stride_b;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return (gchar_ptr)(((uint64_t)hi << 32) | lo);
}

__device__ inline double cgs_load(gchar_ptr base, uint32_t off) {
  return *(const __attribute__((address_space(1))) double*)(base + off);
}

}  // namespace fpc
