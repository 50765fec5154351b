// FGMRES kernels: multi-dot products with fixed-order (deterministic)
// reductions, multi-axpy, scaling, and the small Hessenberg / Givens /
// triangular-solve steps, all on the device.
#include "fpc_apply.hpp"

namespace fpc {

namespace {

constexpr int DT = 256;

__device__ inline double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Partials of <V_i, w> for all i: block b takes rows [b * DT * MR, (b+1) *
// DT * MR), thread t rows b * DT * MR + t + DT * r (r < MR), whose w values
// stay in registers while the vectors stream by, four vectors at a time; one
// partial per block and vector (the four wavefronts added in order),
// part[i * nblocks + b].
constexpr int MR = 4;

__global__ __launch_bounds__(DT) void k_mdot_rows(const double* __restrict__ V,
                                                  int64_t ldv, int nv,
                                                  const double* __restrict__ w,
                                                  int64_t n,
                                                  double* __restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.x * (DT * MR) + threadIdx.x;
  double wv[MR];
#pragma unroll
  for (int r = 0; r < MR; ++r) {
    const int64_t k = r0 + (int64_t)DT * r;
    wv[r] = k < n ? w[k] : 0.0;
  }
  __shared__ double red[4][4];
  const int wave = threadIdx.x >> 6;
  for (int i0 = 0; i0 < nv; i0 += 4) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (i0 + q < nv) {
        const double* __restrict__ v = V + (int64_t)(i0 + q) * ldv;
#pragma unroll
        for (int r = 0; r < MR; ++r) {
          const int64_t k = r0 + (int64_t)DT * r;
          if (k < n) acc[q] += v[k] * wv[r];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double t = wsum(acc[q]);
      if ((threadIdx.x & 63) == 0) red[wave][q] = t;
    }
    __syncthreads();
    if (threadIdx.x < 4 && i0 + (int)threadIdx.x < nv) {
      const int q = threadIdx.x;
      part[(int64_t)(i0 + q) * gridDim.x + blockIdx.x] =
          (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(DT) void k_mdot_reduce(const double* __restrict__ part,
                                                    int np, double* __restrict__ out) {
  __shared__ double sh[DT / 64];
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int k = threadIdx.x; k < np; k += DT) acc += part[(int64_t)i * np + k];
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < DT / 64; ++q) t += sh[q];
    out[i] = t;
  }
}

__global__ __launch_bounds__(DT) void k_maxpy(const double* __restrict__ V,
                                              int64_t ldv, int nv,
                                              const double* __restrict__ h,
                                              double* __restrict__ w, int64_t n) {
  __shared__ double hs[kMaxKrylov];
  if ((int)threadIdx.x < nv) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  for (int64_t k = (int64_t)blockIdx.x * DT + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * DT) {
    double acc = w[k];
    for (int i = 0; i < nv; ++i) acc -= hs[i] * V[(int64_t)i * ldv + k];
    w[k] = acc;
  }
}

// Classical Gram-Schmidt passes over the rows of one grid: block b owns the
// rows b * DT + t + q * G * DT (G = gridDim.x); each thread keeps its partial
// sums for all vectors in registers (NV >= nv, a compile-time bound) and the
// block adds them at the end, wavefronts in order: one partial per block and
// output, part[i * G + b].
template <int NV>
__device__ inline void block_partials(const double (&acc)[NV], int nv,
                                      double* __restrict__ part,
                                      bool has_extra = false,
                                      double extra = 0.0) {
  __shared__ double red[DT / 64][NV + 1];
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i)
    if (i < nv) {
      const double t = wsum(acc[i]);
      if ((threadIdx.x & 63) == 0) red[wave][i] = t;
    }
  if (has_extra) {
    const double t = wsum(extra);
    if ((threadIdx.x & 63) == 0) red[wave][nv] = t;
  }
  __syncthreads();
  if ((int)threadIdx.x < nv + (has_extra ? 1 : 0)) {
    const int i = threadIdx.x;
    part[(int64_t)i * gridDim.x + blockIdx.x] =
        (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
  }
}

// <V_i, w> for i < nv and, as output nv, <w, w>.
template <int NV>
__global__ __launch_bounds__(DT) void k_cgs_dot(const double* __restrict__ V,
                                                int64_t ldv, int nv,
                                                const double* __restrict__ w,
                                                int64_t n,
                                                double* __restrict__ part) {
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  double ww = 0.0;
  const uint64_t stride = (uint64_t)ldv * sizeof(double);
  for (uint32_t k = blockIdx.x * DT + threadIdx.x; k < (uint64_t)n;
       k += gridDim.x * DT) {
    const double wk = w[k];
    const uint32_t off = k * (uint32_t)sizeof(double);
    // re-derive the vector bases each row (scalar arithmetic) instead of
    // holding nv of them live across the loop
    uint64_t st = stride;
    asm volatile("" : "+s"(st));
    // every slot loads (slots beyond nv repeat the last vector, whose rows
    // are in cache, and their sums are dropped): a load under a condition
    // would be waited for before the next one is issued
    double v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i)
      v[i] = cgs_load(cgs_base(V, st, i, nv), off);
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += v[i] * wk;
    ww += wk * wk;
  }
  block_partials<NV>(acc, nv, part, true, ww);
}

// w <- w - sum_i h_i V_i, then <V_i, w> with the updated w: the rows of the
// nv vectors stay in registers between the two uses, so the basis is read
// once.  The update adds in the order of k_maxpy, so w is the same.
template <int NV>
__global__ __launch_bounds__(DT) void k_cgs_axpy_dot(
    const double* __restrict__ V, int64_t ldv, int nv,
    const double* __restrict__ h, double* __restrict__ w, int64_t n,
    double* __restrict__ part) {
  __shared__ double hs[NV];
  if ((int)threadIdx.x < NV) hs[threadIdx.x] = (int)threadIdx.x < nv ? h[threadIdx.x] : 0.0;
  __syncthreads();
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const uint64_t stride = (uint64_t)ldv * sizeof(double);
  for (uint32_t k = blockIdx.x * DT + threadIdx.x; k < (uint64_t)n;
       k += gridDim.x * DT) {
    const uint32_t off = k * (uint32_t)sizeof(double);
    // the coefficients are read from LDS where they are used and the vector
    // bases re-derived each row, so that neither occupies nv registers
    // across the loop
    uint64_t st = stride;
    asm volatile("" : "+s"(st)::"memory");
    // unconditional loads as in k_cgs_dot; hs is zero beyond nv
    double v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i)
      v[i] = cgs_load(cgs_base(V, st, i, nv), off);
    double wk = w[k];
#pragma unroll
    for (int i = 0; i < NV; ++i) wk -= hs[i] * v[i];
    w[k] = wk;
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += v[i] * wk;
  }
  block_partials<NV>(acc, nv, part);
}

// w <- w - sum_i h_i V_i and the partial of <w, w> (one output).
__global__ __launch_bounds__(DT) void k_cgs_axpy_norm(
    const double* __restrict__ V, int64_t ldv, int nv,
    const double* __restrict__ h, double* __restrict__ w, int64_t n,
    double* __restrict__ part) {
  __shared__ double hs[kMaxKrylov];
  if ((int)threadIdx.x < nv) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  double acc[1] = {0.0};
  for (int64_t k = (int64_t)blockIdx.x * DT + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * DT) {
    double wk = w[k];
    for (int i = 0; i < nv; ++i) wk -= hs[i] * V[(int64_t)i * ldv + k];
    w[k] = wk;
    acc[0] += wk * wk;
  }
  block_partials<1>(acc, 1, part);
}

// ---- Gram-Schmidt twice with the second pass delayed by one step (DCGS2,
// Swirydowicz, Langou, Ananthan, Yang and Thomas, Numer. Linear Algebra
// Appl. 2021; Bielich et al., Parallel Comput. 2022).  Step j holds the
// final orthonormal V_0 .. V_{j-1} and, in slot j, u_j: the remainder of
// step j-1's first projection, not normalized.  One pass gives
// <V_i, u_j> and <V_i, w> for i <= j (slot j included, so <u, u> and
// <u, w> come with them); a second pass writes v_j = (u_j - sum a_i V_i) /
// rho_j and u_{j+1} = w - sum b_i V_i - h_j v_j.  The correction a of u_j is
// the second projection of step j-1, so Hessenberg column j-1 is final one
// step late.

// Block partials of two per-vector sums (outputs ou + i and ow + i, i <
// cnt) and optionally one extra (output oe), wavefronts added in order.
template <int NV, bool TWO>
__device__ inline void block_partials2(const double (&au)[NV],
                                       const double (&aw)[NV], int cnt,
                                       double* __restrict__ part, int ou,
                                       int ow, bool has_extra, double extra,
                                       int oe) {
  __shared__ double red[DT / 64][2 * NV + 1];
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i)
    if (i < cnt) {
      const double t = wsum(au[i]);
      if ((threadIdx.x & 63) == 0) red[wave][i] = t;
      if (TWO) {
        const double t2 = wsum(aw[i]);
        if ((threadIdx.x & 63) == 0) red[wave][NV + i] = t2;
      }
    }
  if (has_extra) {
    const double t = wsum(extra);
    if ((threadIdx.x & 63) == 0) red[wave][2 * NV] = t;
  }
  __syncthreads();
  const int G = gridDim.x;
  const int t = threadIdx.x;
  auto sum4 = [&](int q) {
    return (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
  };
  if (t < cnt) part[(int64_t)(ou + t) * G + blockIdx.x] = sum4(t);
  if (TWO && t >= NV && t < NV + cnt)
    part[(int64_t)(ow + t - NV) * G + blockIdx.x] = sum4(t);
  if (has_extra && t == 2 * NV) part[(int64_t)oe * G + blockIdx.x] = sum4(t);
}

// Partials of <V_{i0+i}, u> (output i0 + i) and, with W, <V_{i0+i}, w>
// (output nv + i0 + i) for i < cnt; with EXTRA also <w, w> (output 2 nv).
template <int NV, bool W>
__global__ __launch_bounds__(DT) void k_dcgs_dot(
    const double* __restrict__ V, int64_t ldv, int i0, int cnt, int nv,
    const double* __restrict__ u, const double* __restrict__ w, int64_t n,
    bool extra, double* __restrict__ part) {
  double au[NV], aw[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) au[i] = aw[i] = 0.0;
  double ww = 0.0;
  const double* Vc = V + (int64_t)i0 * ldv;
  const uint64_t stride = (uint64_t)ldv * sizeof(double);
  for (uint32_t k = blockIdx.x * DT + threadIdx.x; k < (uint64_t)n;
       k += gridDim.x * DT) {
    const uint32_t off = k * (uint32_t)sizeof(double);
    const double uk = u[k];
    const double wk = W ? w[k] : 0.0;
    uint64_t st = stride;
    asm volatile("" : "+s"(st));
    double v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = cgs_load(cgs_base(Vc, st, i, cnt), off);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      au[i] += v[i] * uk;
      if (W) aw[i] += v[i] * wk;
    }
    ww += wk * wk;
  }
  block_partials2<NV, W>(au, aw, cnt, part, i0, nv + i0, W && extra, ww,
                         2 * nv);
}

// v_j = (u_j - sum_{i<j} a_i V_i) / rho into slot j and u_{j+1} = w -
// sum_{i<j} b_i V_i - h_j v_j into slot j + 1, with the partials of
// <u_{j+1}, u_{j+1}>.  a = D[0 .. j-1], b = P[0 .. j-1], h_j = P[j], rho =
// scal[0] (v_j = 0 when rho = 0).  For j = 0 the sums are empty.
template <int NV>
__global__ __launch_bounds__(DT) void k_dcgs_update(
    double* V, int64_t ldv, int j, const double* __restrict__ D,
    const double* __restrict__ P, const double* __restrict__ scal,
    const double* __restrict__ w, int64_t n, double* __restrict__ part) {
  __shared__ double2 ab[NV];
  if ((int)threadIdx.x < NV)
    ab[threadIdx.x] = (int)threadIdx.x < j
                          ? make_double2(D[threadIdx.x], P[threadIdx.x])
                          : make_double2(0.0, 0.0);
  __syncthreads();
  const double rho = scal[0];
  const double hj = P[j];
  double* uj = V + (int64_t)j * ldv;
  double* un = V + (int64_t)(j + 1) * ldv;
  const int cnt = j > 0 ? j : 1;  // j = 0: slot 0 loaded with weight 0
  const uint64_t stride = (uint64_t)ldv * sizeof(double);
  double acc[1] = {0.0};
  // rows from the last one down: the dot pass that precedes this one walked
  // them upwards, so the rows it read last are still in the last-level cache
  for (uint32_t kk = blockIdx.x * DT + threadIdx.x; kk < (uint64_t)n;
       kk += gridDim.x * DT) {
    const uint32_t k = (uint32_t)n - 1 - kk;
    const uint32_t off = k * (uint32_t)sizeof(double);
    uint64_t st = stride;
    asm volatile("" : "+s"(st)::"memory");
    double v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = cgs_load(cgs_base(V, st, i, cnt), off);
    double t = uj[k];
    double s = w[k];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double2 c = ab[i];
      t -= c.x * v[i];
      s -= c.y * v[i];
    }
    const double vj = rho != 0.0 ? t / rho : 0.0;
    s -= hj * vj;
    uj[k] = vj;
    un[k] = s;
    acc[0] += s * s;
  }
  block_partials<1>(acc, 1, part);
}

// Applies the rotations 0 .. c-1 (staged in LDS: rc, rs) to col[0 .. c+1]
// (LDS), forms rotation c and returns the residual estimate |g_{c+1}| it
// gives; with commit, also stores the rotation, column c of H and the
// updated g.  Caller: one thread.
__device__ inline double givens_col(double* col, const double* rc,
                                    const double* rs, int c, double* H,
                                    int ldh, double* cs, double* sn, double* g,
                                    bool commit) {
  for (int i = 0; i < c; ++i) {
    const double t = rc[i] * col[i] + rs[i] * col[i + 1];
    col[i + 1] = -rs[i] * col[i] + rc[i] * col[i + 1];
    col[i] = t;
  }
  const double rho = hypot(col[c], col[c + 1]);
  const double cc = rho != 0.0 ? col[c] / rho : 1.0;
  const double ss = rho != 0.0 ? col[c + 1] / rho : 0.0;
  const double gc = g[c];
  if (commit) {
    cs[c] = cc;
    sn[c] = ss;
    col[c] = rho;
    col[c + 1] = 0.0;
    g[c + 1] = -ss * gc;
    g[c] = cc * gc;
    for (int i = 0; i <= c + 1; ++i) H[(int64_t)i * ldh + c] = col[i];
  }
  return fabs(ss * gc);
}

// After the dot pass over nv = j + 1 vectors (slot j = u_j included):
// rho_j = sqrt(<u,u> - |a|^2) (1 for j = 0, whose u_0 is normalized) into
// scal[0]; with fin, Hessenberg column j - 1 made final (P + a, subdiagonal
// rho_j), rotated and committed, its estimate in scal[5], ctrl[0] = 2 if
// rho_j = 0; with fresh, the first projection of column j into P (b, then
// h_j = (<u,w> - a.b) / rho_j) and <w, w> into scal[6].
__global__ __launch_bounds__(64) void k_dcgs_finish(
    const double* __restrict__ D, int nv, int fin, int fresh, double* H,
    int ldh, double* cs, double* sn, double* g, double* P, double* scal,
    int* ctrl) {
  __shared__ double col[kMaxKrylov + 2], rc[kMaxKrylov], rs[kMaxKrylov];
  const int j = nv - 1;
  const int lane = threadIdx.x;
  fin = fin && j > 0;
  double aa = 0.0, ab = 0.0;
  for (int i = lane; i < j; i += 64) {
    const double a = D[i];
    aa += a * a;
    if (fresh) ab += a * D[nv + i];
    if (fin) col[i] = P[i] + a;
  }
  if (fin)
    for (int i = lane; i < j - 1; i += 64) {
      rc[i] = cs[i];
      rs[i] = sn[i];
    }
  aa = wsum(aa);
  ab = wsum(ab);
  __syncthreads();
  if (lane == 0) {
    const double r2 = D[j] - aa;
    const double rho = j == 0 ? 1.0 : (r2 > 0.0 ? sqrt(r2) : 0.0);
    scal[0] = rho;
    int code = 0;
    if (fin) {
      col[j] = rho;
      scal[5] = givens_col(col, rc, rs, j - 1, H, ldh, cs, sn, g, true);
      if (rho == 0.0) code = 2;
    }
    ctrl[0] = code;
    scal[7] = code;
    if (fresh) {
      P[j] = rho != 0.0 ? (D[nv + j] - ab) / rho : 0.0;
      scal[6] = D[2 * nv];
    }
  }
  __syncthreads();
  if (fresh)
    for (int i = lane; i < j; i += 64) P[i] = D[nv + i];
}

// After the update pass: <u_{j+1}, u_{j+1}> reduced from the partials
// (nu_j = its root), the provisional column j (P, subdiagonal nu_j) rotated
// for an estimate of the residual into scal[1].  If nu_j <= 1e-14 |w| (w
// before the projections) the step breaks down: the column is committed as
// it is and ctrl[0] = 1.  Nothing is done if the finish step flagged a
// breakdown.
__global__ __launch_bounds__(DT) void k_dcgs_peek(
    const double* __restrict__ part, int np, double* H, int ldh, double* cs,
    double* sn, double* g, const double* __restrict__ P, int j, double* scal,
    int* ctrl) {
  __shared__ double sh[DT / 64];
  __shared__ double col[kMaxKrylov + 2], rc[kMaxKrylov], rs[kMaxKrylov];
  double acc = 0.0;
  for (int k = threadIdx.x; k < np; k += DT) acc += part[k];
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  for (int i = threadIdx.x; i <= j; i += DT) col[i] = P[i];
  for (int i = threadIdx.x; i < j; i += DT) {
    rc[i] = cs[i];
    rs[i] = sn[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double nu2 = 0.0;
    for (int q = 0; q < DT / 64; ++q) nu2 += sh[q];
    if (ctrl[0] == 2) return;
    const double nu = sqrt(fmax(nu2, 0.0));
    const double w0 = sqrt(fmax(scal[6], 0.0));
    const bool bd = !(nu > 1e-14 * w0);
    col[j + 1] = nu;
    const double est = givens_col(col, rc, rs, j, H, ldh, cs, sn, g, bd);
    scal[1] = est;
    if (bd) {
      scal[5] = est;
      ctrl[0] = 1;
      scal[7] = 1.0;
    }
  }
}

__global__ void k_scale_inv(const double* __restrict__ x,
                            const double* __restrict__ scal,
                            double* __restrict__ y, int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double s = scal[0];
  y[k] = (s != 0.0) ? x[k] / s : 0.0;
}

__global__ void k_axpby(double a, const double* __restrict__ x, double b,
                        double* __restrict__ y, int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  y[k] = (b == 0.0) ? a * x[k] : a * x[k] + b * y[k];
}

// One Arnoldi column: h = h1 + h2 and the new subdiagonal |w|, the previous
// Givens rotations applied to it, the new rotation and the updated residual
// estimate.  The wavefront stages the column and the rotations in LDS, so
// the sequential rotation loop of lane 0 waits on LDS rather than memory.
__global__ __launch_bounds__(64) void k_gmres_step(
    double* H, int ldh, double* cs, double* sn, double* g, const double* h1,
    const double* h2, const double* nrm2, const double* nrm2_before, int j,
    double* scal, int* ctrl) {
  __shared__ double col[kMaxKrylov + 1], c_s[kMaxKrylov], s_s[kMaxKrylov];
  for (int i = threadIdx.x; i <= j; i += 64) {
    col[i] = h1[i] + h2[i];
    if (i < j) {
      c_s[i] = cs[i];
      s_s[i] = sn[i];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double hn = sqrt(fmax(nrm2[0], 0.0));
    const double w0 = sqrt(fmax(nrm2_before[0], 0.0));
    col[j + 1] = hn;
    const int breakdown = !(hn > 1e-14 * w0);
    scal[0] = breakdown ? 0.0 : hn;
    for (int i = 0; i < j; ++i) {
      const double t = c_s[i] * col[i] + s_s[i] * col[i + 1];
      col[i + 1] = -s_s[i] * col[i] + c_s[i] * col[i + 1];
      col[i] = t;
    }
    const double rho = hypot(col[j], col[j + 1]);
    const double c = rho != 0.0 ? col[j] / rho : 1.0;
    const double sgn = rho != 0.0 ? col[j + 1] / rho : 0.0;
    cs[j] = c;
    sn[j] = sgn;
    col[j] = rho;
    col[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sgn * gj;
    g[j] = c * gj;
    scal[1] = fabs(sgn * gj);
    ctrl[0] = breakdown;
    scal[7] = breakdown;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += 64) H[(int64_t)i * ldh + j] = col[i];
}

__global__ void k_gmres_init(double* g, int m, const double* beta2,
                             double* scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double beta = sqrt(fmax(beta2[0], 0.0));
  for (int i = 0; i <= m; ++i) g[i] = 0.0;
  g[0] = beta;
  scal[0] = beta;
  scal[1] = beta;
}

__global__ void k_trisolve(const double* H, int ldh, const double* g,
                           double* y, int k) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int q = i + 1; q < k; ++q) s -= H[(int64_t)i * ldh + q] * y[q];
    y[i] = s / H[(int64_t)i * ldh + i];
  }
}

__global__ void k_sqrt(const double* in, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = sqrt(fmax(in[0], 0.0));
}

}  // namespace

// Blocks of the Gram-Schmidt passes: enough to fill the chip at 1 024, one
// per 256 rows below that.
constexpr int64_t kCgsBlocks = 1024;
// Largest vector count whose rows the fused axpy + dot pass keeps in
// registers (two arrays of NV doubles per thread).
constexpr int kCgsFusedMax = 48;
int64_t cgs_blocks(int64_t n) {
  return std::max<int64_t>(std::min<int64_t>((n + DT - 1) / DT, kCgsBlocks), 1);
}

int64_t mdot_partials(int64_t n, int nv) {
  const int64_t nb = std::max<int64_t>((n + DT * MR - 1) / (DT * MR), 1);
  return (int64_t)nv * std::max(nb, cgs_blocks(n));
}

void mdot(const double* V, int64_t ldv, int nv, const double* w, int64_t n,
          double* partials, double* out, hipStream_t s) {
  if (nv <= 0) return;
  const int64_t nb = std::max<int64_t>((n + DT * MR - 1) / (DT * MR), 1);
  k_mdot_rows<<<(unsigned)nb, DT, 0, s>>>(V, ldv, nv, w, n, partials);
  FPC_LAUNCH_CHECK();
  k_mdot_reduce<<<nv, DT, 0, s>>>(partials, (int)nb, out);
  FPC_LAUNCH_CHECK();
}

#define FPC_CGS_BUCKETS(X) X(8) X(16) X(24) X(32) X(40) X(48) X(56) X(64)

// The passes address a vector's rows by 32-bit byte offsets.
constexpr int64_t kCgsMaxRows = int64_t(1) << 29;

void cgs_dot(const double* V, int64_t ldv, int nv, const double* w, int64_t n,
             double* partials, double* out, hipStream_t s) {
  if (nv < 1 || nv > kMaxKrylov) throw Error(FPC_ERR_ARG, "cgs_dot: vector count");
  if (n >= kCgsMaxRows) {
    mdot(V, ldv, nv, w, n, partials, out, s);
    mdot(w, 0, 1, w, n, partials, out + nv, s);
    return;
  }
  const int64_t G = cgs_blocks(n);
  switch ((nv + 7) / 8) {
#define FPC_CASE(B)                                                          \
  case B / 8:                                                                \
    k_cgs_dot<B><<<(unsigned)G, DT, 0, s>>>(V, ldv, nv, w, n, partials);     \
    break;
    FPC_CGS_BUCKETS(FPC_CASE)
#undef FPC_CASE
  }
  FPC_LAUNCH_CHECK();
  k_mdot_reduce<<<nv + 1, DT, 0, s>>>(partials, (int)G, out);
  FPC_LAUNCH_CHECK();
}

void cgs_axpy_dot(const double* V, int64_t ldv, int nv, const double* h,
                  double* w, int64_t n, double* partials, double* out,
                  hipStream_t s) {
  if (nv < 1 || nv > kMaxKrylov) throw Error(FPC_ERR_ARG, "cgs_axpy_dot: vector count");
  if (nv > kCgsFusedMax || n >= kCgsMaxRows) {
    // beyond the register budget: the two passes separately
    maxpy(V, ldv, nv, h, w, n, s);
    mdot(V, ldv, nv, w, n, partials, out, s);
    return;
  }
  const int64_t G = cgs_blocks(n);
  switch ((nv + 7) / 8) {
#define FPC_CASE(B)                                                        \
  case B / 8:                                                              \
    if constexpr (B <= kCgsFusedMax)                                       \
      k_cgs_axpy_dot<B><<<(unsigned)G, DT, 0, s>>>(V, ldv, nv, h, w, n,    \
                                                  partials);              \
    break;
    FPC_CGS_BUCKETS(FPC_CASE)
#undef FPC_CASE
  }
  FPC_LAUNCH_CHECK();
  k_mdot_reduce<<<nv, DT, 0, s>>>(partials, (int)G, out);
  FPC_LAUNCH_CHECK();
}

void cgs_axpy_norm(const double* V, int64_t ldv, int nv, const double* h,
                   double* w, int64_t n, double* partials, double* out,
                   hipStream_t s) {
  if (nv < 1 || nv > kMaxKrylov) throw Error(FPC_ERR_ARG, "cgs_axpy_norm: vector count");
  const int64_t G = cgs_blocks(n);
  k_cgs_axpy_norm<<<(unsigned)G, DT, 0, s>>>(V, ldv, nv, h, w, n, partials);
  FPC_LAUNCH_CHECK();
  k_mdot_reduce<<<1, DT, 0, s>>>(partials, (int)G, out);
  FPC_LAUNCH_CHECK();
}

bool dcgs_supported(int64_t n) { return n < kCgsMaxRows; }

// Largest vector count of one dot-pass launch (two sums per vector held in
// registers); more vectors take a second launch that reads u and w again.
constexpr int kDcgsChunk = 32;

void dcgs_dot(const double* V, int64_t ldv, int nv, const double* u,
              const double* w, int64_t n, double* partials, double* D,
              hipStream_t s) {
  if (nv < 1 || nv > kMaxKrylov || !dcgs_supported(n))
    throw Error(FPC_ERR_ARG, "dcgs_dot: vector count or length");
  const int64_t G = cgs_blocks(n);
  for (int i0 = 0; i0 < nv; i0 += kDcgsChunk) {
    const int cnt = std::min(kDcgsChunk, nv - i0);
    const bool extra = i0 == 0;
    switch ((cnt + 7) / 8) {
#define FPC_CASE(B)                                                          \
  case B / 8:                                                                \
    if constexpr (B <= kDcgsChunk) {                                         \
      if (w)                                                                 \
        k_dcgs_dot<B, true><<<(unsigned)G, DT, 0, s>>>(                      \
            V, ldv, i0, cnt, nv, u, w, n, extra, partials);                  \
      else                                                                   \
        k_dcgs_dot<B, false><<<(unsigned)G, DT, 0, s>>>(                     \
            V, ldv, i0, cnt, nv, u, w, n, extra, partials);                  \
    }                                                                        \
    break;
      FPC_CGS_BUCKETS(FPC_CASE)
#undef FPC_CASE
    }
    FPC_LAUNCH_CHECK();
  }
  k_mdot_reduce<<<w ? 2 * nv + 1 : nv, DT, 0, s>>>(partials, (int)G, D);
  FPC_LAUNCH_CHECK();
}

void dcgs_finish(const double* D, int nv, bool fin, bool fresh, double* H,
                 int ldh, double* cs, double* sn, double* g, double* P,
                 double* scal, int* ctrl, hipStream_t s) {
  if (nv < 1 || nv > kMaxKrylov) throw Error(FPC_ERR_ARG, "dcgs_finish: j");
  k_dcgs_finish<<<1, 64, 0, s>>>(D, nv, fin ? 1 : 0, fresh ? 1 : 0, H, ldh,
                                 cs, sn, g, P, scal, ctrl);
  FPC_LAUNCH_CHECK();
}

void dcgs_update(double* V, int64_t ldv, int j, const double* D,
                 const double* P, const double* scal, const double* w,
                 int64_t n, double* partials, hipStream_t s) {
  if (j < 0 || j + 1 > kMaxKrylov || !dcgs_supported(n))
    throw Error(FPC_ERR_ARG, "dcgs_update: j or length");
  const int64_t G = cgs_blocks(n);
  switch ((std::max(j, 1) + 7) / 8) {
#define FPC_CASE(B)                                                          \
  case B / 8:                                                                \
    k_dcgs_update<B><<<(unsigned)G, DT, 0, s>>>(V, ldv, j, D, P, scal, w, n, \
                                                partials);                   \
    break;
    FPC_CGS_BUCKETS(FPC_CASE)
#undef FPC_CASE
  }
  FPC_LAUNCH_CHECK();
}

void dcgs_peek(const double* partials, int64_t n, double* H, int ldh,
               double* cs, double* sn, double* g, const double* P, int j,
               double* scal, int* ctrl, hipStream_t s) {
  k_dcgs_peek<<<1, DT, 0, s>>>(partials, (int)cgs_blocks(n), H, ldh, cs, sn,
                               g, P, j, scal, ctrl);
  FPC_LAUNCH_CHECK();
}

void maxpy(const double* V, int64_t ldv, int nv, const double* h, double* w,
           int64_t n, hipStream_t s) {
  if (nv <= 0 || n == 0) return;
  if (nv > kMaxKrylov) throw Error(FPC_ERR_ARG, "maxpy: too many vectors");
  unsigned g = grid_for(n, DT);
  if (g > 8192) g = 8192;
  k_maxpy<<<g, DT, 0, s>>>(V, ldv, nv, h, w, n);
  FPC_LAUNCH_CHECK();
}

void scale_by_inv(const double* x, const double* scal, double* y, int64_t n,
                  hipStream_t s) {
  if (n == 0) return;
  k_scale_inv<<<grid_for(n, 256), 256, 0, s>>>(x, scal, y, n);
  FPC_LAUNCH_CHECK();
}

void axpby(double a, const double* x, double b, double* y, int64_t n,
           hipStream_t s) {
  if (n == 0) return;
  k_axpby<<<grid_for(n, 256), 256, 0, s>>>(a, x, b, y, n);
  FPC_LAUNCH_CHECK();
}

void gmres_step(double* H, int ldh, double* cs, double* sn, double* g,
                const double* h1, const double* h2, const double* nrm2,
                const double* nrm2_before, int j, double* scal, int* ctrl,
                hipStream_t s) {
  if (j + 1 > kMaxKrylov) throw Error(FPC_ERR_ARG, "restart too long");
  k_gmres_step<<<1, 64, 0, s>>>(H, ldh, cs, sn, g, h1, h2, nrm2, nrm2_before,
                                j, scal, ctrl);
  FPC_LAUNCH_CHECK();
}

void gmres_init(double* g, int m, const double* beta2, double* scal,
                hipStream_t s) {
  k_gmres_init<<<1, 64, 0, s>>>(g, m, beta2, scal);
  FPC_LAUNCH_CHECK();
}

void gmres_trisolve(const double* H, int ldh, const double* g, double* y,
                    int k, hipStream_t s) {
  k_trisolve<<<1, 64, 0, s>>>(H, ldh, g, y, k);
  FPC_LAUNCH_CHECK();
}

void sqrt_dev(const double* in, double* out, hipStream_t s) {
  k_sqrt<<<1, 64, 0, s>>>(in, out);
  FPC_LAUNCH_CHECK();
}

}  // namespace fpc
