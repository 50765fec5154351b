// Multi-right-hand-side kernels.  A block of KB right-hand sides is stored
// interleaved: element (n, c) at n * KB + c, so every sparse row is read once
// for all columns and column accesses of a row are contiguous.
#include "fpc_apply.hpp"

namespace fpc {

namespace {

__global__ void k_pack(const double* __restrict__ B, int64_t ldb, int64_t n,
                       int k, int KB, double* __restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * KB) return;
  const int64_t i = t / KB;
  const int c = (int)(t % KB);
  out[t] = c < k ? B[(int64_t)c * ldb + i] : 0.0;
}

__global__ void k_unpack(const double* __restrict__ Xi, int64_t n, int k,
                         int KB, double* __restrict__ X, int64_t ldx) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * k) return;
  const int c = (int)(t / n);
  const int64_t i = t % n;
  X[(int64_t)c * ldx + i] = Xi[i * KB + c];
}

__global__ void k_face_apply_b(const double* __restrict__ hinv,
                               const double* __restrict__ in,
                               double* __restrict__ out, int64_t n_p, int KB,
                               int trans) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_p * KB) return;
  const int64_t K = t / KB;
  const int c = (int)(t % KB);
  const double* h = hinv + K * 9;
  const double a = in[(3 * K) * KB + c], b = in[(3 * K + 1) * KB + c],
               d = in[(3 * K + 2) * KB + c];
  for (int r = 0; r < 3; ++r) {
    const double v = trans ? h[0 * 3 + r] * a + h[1 * 3 + r] * b + h[2 * 3 + r] * d
                           : h[r * 3 + 0] * a + h[r * 3 + 1] * b + h[r * 3 + 2] * d;
    out[(3 * K + r) * KB + c] = v;
  }
}

// y(i, c) = beta y(i, c) + a1 (M1 x1)(i, c) + a2 (M2 x2)(i, c)
__global__ void k_csr_spmv2_b(const int64_t* rp1, const int32_t* c1,
                              const double* v1, const double* x1, double a1,
                              const int64_t* rp2, const int32_t* c2,
                              const double* v2, const double* x2, double a2,
                              double* y, double beta, int64_t nrows, int KB) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * KB) return;
  const int64_t i = t / KB;
  const int c = (int)(t % KB);
  const double s1 = csr_row_sum_col(c1, v1, x1, rp1[i], rp1[i + 1], KB, c);
  double r = a1 * s1;
  if (rp2) {
    const double s2 = csr_row_sum_col(c2, v2, x2, rp2[i], rp2[i + 1], KB, c);
    r += a2 * s2;
  }
  y[t] = (beta == 0.0) ? r : beta * y[t] + r;
}

// level-0 input per right-hand side:
// out(i, c) = (T)(base(i, c) + a1 (M1 x1)(i, c) + a2 (M2 x2)(i, c))
template <typename T>
__global__ void k_to_level_b(T* __restrict__ out, int KB,
                             const double* __restrict__ base,
                             const int64_t* rp1, const int32_t* c1,
                             const double* v1, const double* x1, double a1,
                             const int64_t* rp2, const int32_t* c2,
                             const double* v2, const double* x2, double a2,
                             int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * KB) return;
  const int64_t i = t / KB;
  const int c = (int)(t % KB);
  double r = base ? base[t] : 0.0;
  r += a1 * csr_row_sum_col(c1, v1, x1, rp1[i], rp1[i + 1], KB, c);
  r += a2 * csr_row_sum_col(c2, v2, x2, rp2[i], rp2[i + 1], KB, c);
  out[t] = (T)r;
}

template <typename T>
__global__ void k_from_level_b(const T* __restrict__ xo, int64_t n, int KB,
                               double* __restrict__ vu) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * KB) return;
  const int64_t i = t / KB;
  const int c = (int)(t % KB);
  vu[t] = (double)xo[i * KB + c];
}

__global__ void k_tface_b(const int64_t* __restrict__ rp,
                          const int32_t* __restrict__ col,
                          const double* __restrict__ val,
                          const double* __restrict__ vu,
                          const double* __restrict__ t_t,
                          const double* __restrict__ hinv,
                          double* __restrict__ v_t, int64_t n_p, int KB) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_p * KB) return;
  const int64_t K = t / KB;
  const int c = (int)(t % KB);
  double s[3];
  for (int r = 0; r < 3; ++r) {
    const int64_t row = 3 * K + r;
    s[r] = csr_row_sum_col(col, val, vu, rp[row], rp[row + 1], KB, c);
  }
  const double* h = hinv + K * 9;
  for (int r = 0; r < 3; ++r)
    v_t[(3 * K + r) * KB + c] = -t_t[(3 * K + r) * KB + c] +
                                h[r * 3] * s[0] + h[r * 3 + 1] * s[1] +
                                h[r * 3 + 2] * s[2];
}

// ------------------------------------------------------------- Krylov
constexpr int BT = 256;

// grid (chunks, nv); block = (BT / KB) row lanes x KB columns
__global__ __launch_bounds__(BT) void k_bmdot_partial(
    const double* __restrict__ V, int64_t ldv, const double* __restrict__ W,
    int64_t n, int KB, double* __restrict__ part) {
  __shared__ double sh[BT];
  const int i = blockIdx.y;
  const int rl = threadIdx.x / KB, c = threadIdx.x % KB;
  const int nrl = BT / KB;
  const double* __restrict__ v = V + (int64_t)i * ldv;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t a = (int64_t)blockIdx.x * chunk;
  const int64_t b = min(n, a + chunk);
  double acc = 0.0;
  for (int64_t r = a + rl; r < b; r += nrl) acc += v[r * KB + c] * W[r * KB + c];
  sh[threadIdx.x] = acc;
  __syncthreads();
  if (rl == 0) {
    double t = 0.0;
    for (int q = 0; q < nrl; ++q) t += sh[q * KB + c];
    part[((int64_t)i * gridDim.x + blockIdx.x) * KB + c] = t;
  }
}

// out(i, c) = sum_q part[(i * np + q) * KB + c]: block i, thread (ql, c)
// = (tid / KB, tid % KB) adds every nql-th partial, then the nql sums are
// added in order.
__global__ __launch_bounds__(BT) void k_bmdot_reduce(
    const double* __restrict__ part, int np, int KB, double* __restrict__ out) {
  __shared__ double sh[BT];
  const int i = blockIdx.x;
  const int ql = threadIdx.x / KB, c = threadIdx.x % KB, nql = BT / KB;
  double t = 0.0;
  if (ql < nql)
    for (int q = ql; q < np; q += nql) t += part[((int64_t)i * np + q) * KB + c];
  sh[threadIdx.x] = t;
  __syncthreads();
  if ((int)threadIdx.x < KB) {
    double a = 0.0;
    for (int q = 0; q < nql; ++q) a += sh[q * KB + threadIdx.x];
    out[(int64_t)i * KB + threadIdx.x] = a;
  }
}

// W(n, c) -= sum_i sgn * h(i, c) V_i(n, c)
__global__ __launch_bounds__(BT) void k_bmaxpy(const double* __restrict__ V,
                                               int64_t ldv, int nv,
                                               const double* __restrict__ h,
                                               double* __restrict__ W,
                                               int64_t n, int KB) {
  __shared__ double hs[kMaxKrylov * 32];
  for (int q = threadIdx.x; q < nv * KB; q += BT) hs[q] = h[q];
  __syncthreads();
  const int64_t tot = n * KB;
  for (int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x; t < tot;
       t += (int64_t)gridDim.x * BT) {
    const int c = (int)(t % KB);
    double acc = W[t];
    for (int i = 0; i < nv; ++i) acc -= hs[i * KB + c] * V[(int64_t)i * ldv + t];
    W[t] = acc;
  }
}

// Batched classical Gram-Schmidt passes (the three passes of the single
// right-hand-side solve, per column).  Element t = r * KB + c of a vector
// (row r, column c); thread (rl, c) = (tid / KB, tid % KB) of block b takes
// rows r = b * nrl + rl + q * G * nrl with nrl = BT / KB, and keeps one
// partial per vector in registers; the block adds them per column at the
// end, part[(o * G + b) * KB + c] for output o.
__device__ inline double bwsum_cols(double* sh, double val, int KB, int nrl) {
  // column sums over the block's row lanes; valid in threads tid < KB
  __syncthreads();
  sh[threadIdx.x] = val;
  __syncthreads();
  double t = 0.0;
  if ((int)threadIdx.x < KB)
    for (int q = 0; q < nrl; ++q) t += sh[q * KB + threadIdx.x];
  return t;
}

template <int NV>
__device__ inline void bblock_partials(const double (&acc)[NV], int nv,
                                       bool has_extra, double extra, int KB,
                                       double* __restrict__ part) {
  __shared__ double sh[BT];
  const int rl = threadIdx.x / KB, nrl = BT / KB;
  const bool lane_ok = rl < nrl;
#pragma unroll
  for (int o = 0; o <= NV; ++o) {
    if (o > nv || (o == nv && !has_extra)) break;
    double val = 0.0;
    if (o < NV) val = acc[o];
    if (o == nv) val = extra;
    const double t = bwsum_cols(sh, lane_ok ? val : 0.0, KB, nrl);
    if ((int)threadIdx.x < KB)
      part[((int64_t)o * gridDim.x + blockIdx.x) * KB + threadIdx.x] = t;
  }
}

// <V_i, W> per column for i < nv and, as output nv, <W, W>.
template <int NV>
__global__ __launch_bounds__(BT) void k_bcgs_dot(const double* __restrict__ V,
                                                 int64_t ldv, int nv,
                                                 const double* __restrict__ W,
                                                 int64_t n, int KB,
                                                 double* __restrict__ part) {
  const int rl = threadIdx.x / KB, c = threadIdx.x % KB, nrl = BT / KB;
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  double ww = 0.0;
  if (rl < nrl) {
    const uint64_t stride = (uint64_t)ldv * sizeof(double);
    for (int64_t r = (int64_t)blockIdx.x * nrl + rl; r < n;
         r += (int64_t)gridDim.x * nrl) {
      const uint32_t t = (uint32_t)(r * KB + c);
      const double wk = W[t];
      const uint32_t off = t * (uint32_t)sizeof(double);
      uint64_t st = stride;
      asm volatile("" : "+s"(st));
      double v[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] = cgs_load(cgs_base(V, st, i, nv), off);
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += v[i] * wk;
      ww += wk * wk;
    }
  }
  bblock_partials<NV>(acc, nv, true, ww, KB, part);
}

// W -= sum_i h(i, c) V_i, then <V_i, W> per column from the same rows.
template <int NV>
__global__ __launch_bounds__(BT) void k_bcgs_axpy_dot(
    const double* __restrict__ V, int64_t ldv, int nv,
    const double* __restrict__ h, double* __restrict__ W, int64_t n, int KB,
    double* __restrict__ part) {
  __shared__ double hs[NV * 32];
  for (int q = threadIdx.x; q < NV * KB; q += BT) hs[q] = q < nv * KB ? h[q] : 0.0;
  __syncthreads();
  const int rl = threadIdx.x / KB, c = threadIdx.x % KB, nrl = BT / KB;
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  if (rl < nrl) {
    const uint64_t stride = (uint64_t)ldv * sizeof(double);
    for (int64_t r = (int64_t)blockIdx.x * nrl + rl; r < n;
         r += (int64_t)gridDim.x * nrl) {
      const uint32_t t = (uint32_t)(r * KB + c);
      const uint32_t off = t * (uint32_t)sizeof(double);
      // the coefficients are read from LDS where they are used and the
      // vector bases re-derived each row
      uint64_t st = stride;
      asm volatile("" : "+s"(st)::"memory");
      double v[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] = cgs_load(cgs_base(V, st, i, nv), off);
      double wk = W[t];
#pragma unroll
      for (int i = 0; i < NV; ++i) wk -= hs[i * KB + c] * v[i];
      W[t] = wk;
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += v[i] * wk;
    }
  }
  bblock_partials<NV>(acc, nv, false, 0.0, KB, part);
}

// W -= sum_i h(i, c) V_i and the partial of <W, W> per column.
__global__ __launch_bounds__(BT) void k_bcgs_axpy_norm(
    const double* __restrict__ V, int64_t ldv, int nv,
    const double* __restrict__ h, double* __restrict__ W, int64_t n, int KB,
    double* __restrict__ part) {
  __shared__ double hs[kMaxKrylov * 32];
  for (int q = threadIdx.x; q < nv * KB; q += BT) hs[q] = h[q];
  __syncthreads();
  const int rl = threadIdx.x / KB, c = threadIdx.x % KB, nrl = BT / KB;
  double acc[1] = {0.0};
  if (rl < nrl) {
    for (int64_t r = (int64_t)blockIdx.x * nrl + rl; r < n;
         r += (int64_t)gridDim.x * nrl) {
      const int64_t t = r * KB + c;
      double wk = W[t];
      for (int i = 0; i < nv; ++i) wk -= hs[i * KB + c] * V[(int64_t)i * ldv + t];
      W[t] = wk;
      acc[0] += wk * wk;
    }
  }
  bblock_partials<1>(acc, 1, false, 0.0, KB, part);
}

// ---- Batched delayed Gram-Schmidt: the dcgs_* steps of the single solve,
// per column of the interleaved block (element t = r * KB + c), with
// per-column masks: active (column still iterating), pf (its last Hessenberg
// column is final) and, for the finalizing pass, needfin.

// Per-column block partials of two per-vector sums, outputs ou + i and
// ow + i (i < cnt), and optionally an extra one (output oe):
// part[(o * G + b) * KB + c].
template <int NV, bool TWO>
__device__ inline void bblock_partials2(const double (&au)[NV],
                                        const double (&aw)[NV], int cnt,
                                        int ou, int ow, bool has_extra,
                                        double extra, int oe, int KB,
                                        double* __restrict__ part) {
  __shared__ double sh[BT];
  const int rl = threadIdx.x / KB, nrl = BT / KB;
  const bool lane_ok = rl < nrl;
  const int64_t G = gridDim.x;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (i < cnt) {
      double t = bwsum_cols(sh, lane_ok ? au[i] : 0.0, KB, nrl);
      if ((int)threadIdx.x < KB)
        part[((int64_t)(ou + i) * G + blockIdx.x) * KB + threadIdx.x] = t;
      if (TWO) {
        t = bwsum_cols(sh, lane_ok ? aw[i] : 0.0, KB, nrl);
        if ((int)threadIdx.x < KB)
          part[((int64_t)(ow + i) * G + blockIdx.x) * KB + threadIdx.x] = t;
      }
    }
  }
  if (has_extra) {
    const double t = bwsum_cols(sh, lane_ok ? extra : 0.0, KB, nrl);
    if ((int)threadIdx.x < KB)
      part[((int64_t)oe * G + blockIdx.x) * KB + threadIdx.x] = t;
  }
}

// Per column: <V_{i0+i}, U> (output i0 + i) and, with W, <V_{i0+i}, W>
// (output nv + i0 + i), i < cnt; with extra also <W, W> (output 2 nv).
template <int NV, bool WW>
__global__ __launch_bounds__(BT) void k_bdcgs_dot(
    const double* __restrict__ V, int64_t ldv, int i0, int cnt, int nv,
    const double* __restrict__ U, const double* __restrict__ W, int64_t n,
    int KB, bool extra, double* __restrict__ part) {
  const int rl = threadIdx.x / KB, c = threadIdx.x % KB, nrl = BT / KB;
  double au[NV], aw[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) au[i] = aw[i] = 0.0;
  double ww = 0.0;
  const double* Vc = V + (int64_t)i0 * ldv;
  if (rl < nrl) {
    const uint64_t stride = (uint64_t)ldv * sizeof(double);
    for (int64_t r = (int64_t)blockIdx.x * nrl + rl; r < n;
         r += (int64_t)gridDim.x * nrl) {
      const uint32_t t = (uint32_t)(r * KB + c);
      const uint32_t off = t * (uint32_t)sizeof(double);
      const double uk = U[t];
      const double wk = WW ? W[t] : 0.0;
      uint64_t st = stride;
      asm volatile("" : "+s"(st));
      double v[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] = cgs_load(cgs_base(Vc, st, i, cnt), off);
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        au[i] += v[i] * uk;
        if (WW) aw[i] += v[i] * wk;
      }
      ww += wk * wk;
    }
  }
  bblock_partials2<NV, WW>(au, aw, cnt, i0, nv + i0, WW && extra, ww, 2 * nv,
                           KB, part);
}

// Per column: v_j = (u_j - sum_{i<j} a_i V_i) / rho into slot j and
// u_{j+1} = W - sum_{i<j} b_i V_i - h_j v_j into slot j + 1, with the
// partials of |u_{j+1}|^2; a(i, c) = D[i KB + c], b(i, c) = P[i KB + c],
// h_j = P[j KB + c] (v_j = 0 where rho = 0).
template <int NV>
__global__ __launch_bounds__(BT) void k_bdcgs_update(
    double* V, int64_t ldv, int j, const double* __restrict__ D,
    const double* __restrict__ P, const double* __restrict__ rho,
    const double* __restrict__ W, int64_t n, int KB,
    double* __restrict__ part) {
  __shared__ double2 ab[NV * 32];
  for (int q = threadIdx.x; q < NV * KB; q += BT) {
    const int i = q / KB;
    ab[q] = i < j ? make_double2(D[q], P[q]) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int rl = threadIdx.x / KB, c = threadIdx.x % KB, nrl = BT / KB;
  const double rc = rho[c];
  const double hj = P[(int64_t)j * KB + c];
  double* uj = V + (int64_t)j * ldv;
  double* un = V + (int64_t)(j + 1) * ldv;
  const int cnt = j > 0 ? j : 1;  // j = 0: slot 0 loaded with weight 0
  double acc[1] = {0.0};
  if (rl < nrl) {
    const uint64_t stride = (uint64_t)ldv * sizeof(double);
    for (int64_t r = (int64_t)blockIdx.x * nrl + rl; r < n;
         r += (int64_t)gridDim.x * nrl) {
      const uint32_t t = (uint32_t)(r * KB + c);
      const uint32_t off = t * (uint32_t)sizeof(double);
      uint64_t st = stride;
      asm volatile("" : "+s"(st)::"memory");
      double v[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] = cgs_load(cgs_base(V, st, i, cnt), off);
      double tu = uj[t];
      double sw = W[t];
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const double2 cf = ab[i * KB + c];
        tu -= cf.x * v[i];
        sw -= cf.y * v[i];
      }
      const double vj = rc != 0.0 ? tu / rc : 0.0;
      sw -= hj * vj;
      uj[t] = vj;
      un[t] = sw;
      acc[0] += sw * sw;
    }
  }
  bblock_partials<1>(acc, 1, false, 0.0, KB, part);
}

// Column c's Givens step on column cc of its Hessenberg matrix (col in
// private memory, rotations read from cs / sn); returns |g_{cc+1}| and,
// with commit, stores the rotation, the column and g.
__device__ inline double bgivens_col(double* col, int cc, double* Hc, int m,
                                     double* csc, double* snc, double* gc,
                                     bool commit) {
  for (int i = 0; i < cc; ++i) {
    const double t = csc[i] * col[i] + snc[i] * col[i + 1];
    col[i + 1] = -snc[i] * col[i] + csc[i] * col[i + 1];
    col[i] = t;
  }
  const double r = hypot(col[cc], col[cc + 1]);
  const double cj = r != 0.0 ? col[cc] / r : 1.0;
  const double sj = r != 0.0 ? col[cc + 1] / r : 0.0;
  const double gj = gc[cc];
  if (commit) {
    csc[cc] = cj;
    snc[cc] = sj;
    col[cc] = r;
    col[cc + 1] = 0.0;
    gc[cc + 1] = -sj * gj;
    gc[cc] = cj * gj;
    for (int i = 0; i <= cc + 1; ++i) Hc[(int64_t)i * m + cc] = col[i];
  }
  return fabs(sj * gj);
}

// After a dot pass over nv = j + 1 vectors (slot j = u_j included), per
// active column: rho_j (1 for j = 0); Hessenberg column j - 1 made final
// when fresh and pf[c] = 0, or when needfin[c] (fresh = 0): estimate in
// sc[KB + c], code 2 where rho_j = 0, pf[c] = 1; with fresh the first
// projection of column j into P, <W, W> into ww[c], pf[c] = 0.  sc[2 KB + c]
// holds the code (0, 1 breakdown at step j, 2).  Inactive columns get rho =
// 0 and a zero projection.
__global__ void k_bdcgs_finish(const double* __restrict__ D, int nv, int fresh,
                               const int* __restrict__ needfin, double* H,
                               int m, double* cs, double* sn, double* g,
                               double* P, double* rho, double* ww, double* sc,
                               int* pf, const int* __restrict__ active,
                               int KB) {
  const int c = threadIdx.x;
  if (c >= KB) return;
  const int j = nv - 1;
  if (!active[c]) {
    if (fresh) {
      rho[c] = 0.0;
      for (int i = 0; i <= j; ++i) P[(int64_t)i * KB + c] = 0.0;
    }
    sc[2 * KB + c] = 0.0;
    return;
  }
  double aa = 0.0, ab = 0.0;
  for (int i = 0; i < j; ++i) {
    const double a = D[(int64_t)i * KB + c];
    aa += a * a;
    if (fresh) ab += a * D[(int64_t)(nv + i) * KB + c];
  }
  const double r2 = D[(int64_t)j * KB + c] - aa;
  const double rh = j == 0 ? 1.0 : (r2 > 0.0 ? sqrt(r2) : 0.0);
  rho[c] = rh;
  int code = 0;
  const bool fin = fresh ? (j > 0 && !pf[c]) : (needfin[c] != 0);
  if (fin && j > 0) {
    double col[kMaxKrylov + 2];
    for (int i = 0; i < j; ++i)
      col[i] = P[(int64_t)i * KB + c] + D[(int64_t)i * KB + c];
    col[j] = rh;
    sc[KB + c] = bgivens_col(col, j - 1, H + (int64_t)c * (m + 1) * m, m,
                             cs + (int64_t)c * m, sn + (int64_t)c * m,
                             g + (int64_t)c * (m + 1), true);
    if (rh == 0.0) code = 2;
    pf[c] = 1;
  }
  if (fresh) {
    P[(int64_t)j * KB + c] =
        rh != 0.0 ? (D[(int64_t)(nv + j) * KB + c] - ab) / rh : 0.0;
    for (int i = 0; i < j; ++i)
      P[(int64_t)i * KB + c] = D[(int64_t)(nv + i) * KB + c];
    ww[c] = D[(int64_t)(2 * nv) * KB + c];
    pf[c] = 0;
  }
  sc[2 * KB + c] = code;
}

// After the update pass: per active column (code != 2) |u_{j+1}|^2 reduced
// from the partials (in the order of k_bmdot_reduce), the provisional column
// j (P, subdiagonal nu_j) rotated for the estimate sc[c]; nu_j <= 1e-14 |W|
// is a breakdown: the column is committed, sc[KB + c] = estimate, code 1,
// pf[c] = 1.
__global__ __launch_bounds__(BT) void k_bdcgs_peek(
    const double* __restrict__ part, int np, double* H, int m, double* cs,
    double* sn, double* g, const double* __restrict__ P, int j,
    const double* __restrict__ ww, double* sc, int* pf,
    const int* __restrict__ active, int KB) {
  __shared__ double sh[BT];
  const int ql = threadIdx.x / KB, c0 = threadIdx.x % KB, nql = BT / KB;
  double t = 0.0;
  if (ql < nql)
    for (int q = ql; q < np; q += nql) t += part[(int64_t)q * KB + c0];
  sh[threadIdx.x] = t;
  __syncthreads();
  const int c = threadIdx.x;
  if (c >= KB || !active[c] || sc[2 * KB + c] == 2.0) return;
  double nu2 = 0.0;
  for (int q = 0; q < nql; ++q) nu2 += sh[q * KB + c];
  const double nu = sqrt(fmax(nu2, 0.0));
  const double w0 = sqrt(fmax(ww[c], 0.0));
  const bool bd = !(nu > 1e-14 * w0);
  double col[kMaxKrylov + 2];
  for (int i = 0; i <= j; ++i) col[i] = P[(int64_t)i * KB + c];
  col[j + 1] = nu;
  const double est = bgivens_col(col, j, H + (int64_t)c * (m + 1) * m, m,
                                 cs + (int64_t)c * m, sn + (int64_t)c * m,
                                 g + (int64_t)c * (m + 1), bd);
  sc[c] = est;
  if (bd) {
    sc[KB + c] = est;
    sc[2 * KB + c] = 1.0;
    pf[c] = 1;
  }
}

__global__ void k_bscale(const double* __restrict__ x,
                         const double* __restrict__ scal, double* __restrict__ y,
                         int64_t n, int KB) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * KB) return;
  const double s = scal[t % KB];
  y[t] = (s != 0.0) ? x[t] / s : 0.0;
}

__global__ void k_bsub(const double* __restrict__ a, double* __restrict__ b,
                       int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) b[t] = a[t] - b[t];
}

// per column c: Givens update of step j (columns with active[c] == 0 keep
// their state); scal[c] = h_{j+1,j} (0 on breakdown / inactive),
// est[c] = |g_{j+1}|, brk[c] = breakdown
__global__ void k_bgmres_step(double* H, double* cs, double* sn, double* g,
                              const double* h1, const double* h2,
                              const double* nrm2, const double* nrm0, int j,
                              int m, int KB, const int* active, double* scal,
                              double* est, int* brk) {
  const int c = threadIdx.x;
  if (c >= KB) return;
  if (!active[c]) {
    scal[c] = 0.0;
    est[c] = 0.0;
    brk[c] = 0;
    return;
  }
  double* Hc = H + (int64_t)c * (m + 1) * m;
  double* csc = cs + c * m;
  double* snc = sn + c * m;
  double* gc = g + c * (m + 1);
  double col[kMaxKrylov + 1];
  for (int i = 0; i <= j; ++i) col[i] = h1[i * KB + c] + h2[i * KB + c];
  const double hn = sqrt(fmax(nrm2[c], 0.0));
  const double w0 = sqrt(fmax(nrm0[c], 0.0));
  col[j + 1] = hn;
  const int breakdown = !(hn > 1e-14 * w0);
  scal[c] = breakdown ? 0.0 : hn;
  for (int i = 0; i < j; ++i) {
    const double t = csc[i] * col[i] + snc[i] * col[i + 1];
    col[i + 1] = -snc[i] * col[i] + csc[i] * col[i + 1];
    col[i] = t;
  }
  const double rho = hypot(col[j], col[j + 1]);
  const double cj = rho != 0.0 ? col[j] / rho : 1.0;
  const double sj = rho != 0.0 ? col[j + 1] / rho : 0.0;
  csc[j] = cj;
  snc[j] = sj;
  col[j] = rho;
  col[j + 1] = 0.0;
  gc[j + 1] = -sj * gc[j];
  gc[j] = cj * gc[j];
  for (int i = 0; i <= j + 1; ++i) Hc[(int64_t)i * m + j] = col[i];
  est[c] = fabs(gc[j + 1]);
  brk[c] = breakdown;
}

__global__ void k_bgmres_init(double* g, int m, int KB, const double* beta2,
                              const int* active, double* scal) {
  const int c = threadIdx.x;
  if (c >= KB) return;
  const double beta = active[c] ? sqrt(fmax(beta2[c], 0.0)) : 0.0;
  double* gc = g + c * (m + 1);
  for (int i = 0; i <= m; ++i) gc[i] = 0.0;
  gc[0] = beta;
  scal[c] = beta;
}

// y(:, c) = R_c^{-1} g_c for the first kc[c] steps; stored y[j * KB + c]
__global__ void k_btrisolve(const double* H, const double* g, double* y,
                            const int* kc, int m, int KB) {
  const int c = threadIdx.x;
  if (c >= KB) return;
  const double* Hc = H + (int64_t)c * (m + 1) * m;
  const double* gc = g + c * (m + 1);
  const int k = kc[c];
  for (int j = 0; j < m; ++j) y[j * KB + c] = 0.0;
  for (int i = k - 1; i >= 0; --i) {
    double s = gc[i];
    for (int q = i + 1; q < k; ++q) s -= Hc[(int64_t)i * m + q] * y[q * KB + c];
    y[i * KB + c] = s / Hc[(int64_t)i * m + i];
  }
}

}  // namespace

void pack_cols(const double* B, int64_t ldb, int64_t n, int k, int KB,
               double* out, hipStream_t s) {
  k_pack<<<grid_for(n * KB, 256), 256, 0, s>>>(B, ldb, n, k, KB, out);
  FPC_LAUNCH_CHECK();
}

void unpack_cols(const double* Xi, int64_t n, int k, int KB, double* X,
                 int64_t ldx, hipStream_t s) {
  k_unpack<<<grid_for(n * k, 256), 256, 0, s>>>(Xi, n, k, KB, X, ldx);
  FPC_LAUNCH_CHECK();
}

void face_apply_b(const double* hinv, const double* in, double* out,
                  int64_t n_p, int KB, int trans, hipStream_t s) {
  if (!n_p) return;
  k_face_apply_b<<<grid_for(n_p * KB, 256), 256, 0, s>>>(hinv, in, out, n_p,
                                                          KB, trans);
  FPC_LAUNCH_CHECK();
}

void csr_spmv2_b(const Csr* m1, const double* x1, double a1, const Csr* m2,
                 const double* x2, double a2, double* y, double beta, int KB,
                 hipStream_t s) {
  if (!m1->nrows) return;
  k_csr_spmv2_b<<<grid_for(m1->nrows * KB, 256), 256, 0, s>>>(
      m1->rowptr.p, m1->col.p, m1->val.p, x1, a1,
      m2 ? m2->rowptr.p : nullptr, m2 ? m2->col.p : nullptr,
      m2 ? m2->val.p : nullptr, x2, a2, y, beta, m1->nrows, KB);
  FPC_LAUNCH_CHECK();
}

template <typename T>
void to_level_b(T* out, int KB, int64_t n, const double* base,
                const Csr& M1, const double* x1, double a1, const Csr& M2,
                const double* x2, double a2, hipStream_t s) {
  if (!n) return;
  k_to_level_b<T><<<grid_for(n * KB, 256), 256, 0, s>>>(
      out, KB, base, M1.rowptr.p, M1.col.p, M1.val.p, x1, a1, M2.rowptr.p,
      M2.col.p, M2.val.p, x2, a2, n);
  FPC_LAUNCH_CHECK();
}
template void to_level_b<double>(double*, int, int64_t, const double*,
                                 const Csr&, const double*, double, const Csr&,
                                 const double*, double, hipStream_t);
template void to_level_b<float>(float*, int, int64_t, const double*,
                                const Csr&, const double*, double, const Csr&,
                                const double*, double, hipStream_t);

template <typename T>
void from_level_b(const T* xo, int64_t n, int KB, double* vu, hipStream_t s) {
  if (!n) return;
  k_from_level_b<T><<<grid_for(n * KB, 256), 256, 0, s>>>(xo, n, KB, vu);
  FPC_LAUNCH_CHECK();
}
template void from_level_b<double>(const double*, int64_t, int, double*,
                                   hipStream_t);
template void from_level_b<float>(const float*, int64_t, int, double*,
                                  hipStream_t);

void tface_b(const Csr& C, const double* vu, const double* t_t,
             const double* hinv, double* v_t, int64_t n_p, int KB,
             hipStream_t s) {
  if (!n_p) return;
  k_tface_b<<<grid_for(n_p * KB, 128), 128, 0, s>>>(
      C.rowptr.p, C.col.p, C.val.p, vu, t_t, hinv, v_t, n_p, KB);
  FPC_LAUNCH_CHECK();
}

void bmdot(const double* V, int64_t ldv, int nv, const double* W, int64_t n,
           int KB, double* part, double* out, hipStream_t s) {
  if (nv <= 0) return;
  dim3 grid(kDotBlocks, nv);
  k_bmdot_partial<<<grid, BT, 0, s>>>(V, ldv, W, n, KB, part);
  FPC_LAUNCH_CHECK();
  k_bmdot_reduce<<<nv, BT, 0, s>>>(part, kDotBlocks, KB, out);
  FPC_LAUNCH_CHECK();
}

// Blocks of the batched Gram-Schmidt passes.
constexpr int64_t kBcgsBlocks = 1024;
// Largest vector count the fused axpy + dot pass keeps in registers.
constexpr int kBcgsFusedMax = 48;

int64_t bcgs_blocks(int64_t n, int KB) {
  const int64_t nrl = BT / KB;
  return std::max<int64_t>(std::min<int64_t>((n + nrl - 1) / nrl, kBcgsBlocks), 1);
}

int64_t bdot_partials(int nv, int KB) {
  return (int64_t)nv * std::max<int64_t>(kDotBlocks, kBcgsBlocks) * KB;
}

// 32-bit element offsets address the vectors of the fused passes
static bool bcgs_fits(int64_t n, int KB) {
  return n * KB < (int64_t(1) << 29);
}

#define FPC_BCGS_BUCKETS(X) X(8) X(16) X(24) X(32) X(40) X(48) X(56) X(64)

void bcgs_dot(const double* V, int64_t ldv, int nv, const double* W, int64_t n,
              int KB, double* part, double* out, hipStream_t s) {
  if (nv < 1 || nv > kMaxKrylov || KB < 1 || KB > 32)
    throw Error(FPC_ERR_ARG, "bcgs_dot size");
  if (!bcgs_fits(n, KB)) {
    bmdot(V, ldv, nv, W, n, KB, part, out, s);
    bmdot(W, 0, 1, W, n, KB, part, out + (int64_t)nv * KB, s);
    return;
  }
  const int64_t G = bcgs_blocks(n, KB);
  switch ((nv + 7) / 8) {
#define FPC_CASE(B)                                                         \
  case B / 8:                                                               \
    k_bcgs_dot<B><<<(unsigned)G, BT, 0, s>>>(V, ldv, nv, W, n, KB, part);   \
    break;
    FPC_BCGS_BUCKETS(FPC_CASE)
#undef FPC_CASE
  }
  FPC_LAUNCH_CHECK();
  k_bmdot_reduce<<<nv + 1, BT, 0, s>>>(part, (int)G, KB, out);
  FPC_LAUNCH_CHECK();
}

void bcgs_axpy_dot(const double* V, int64_t ldv, int nv, const double* h,
                   double* W, int64_t n, int KB, double* part, double* out,
                   hipStream_t s) {
  if (nv < 1 || nv > kMaxKrylov || KB < 1 || KB > 32)
    throw Error(FPC_ERR_ARG, "bcgs_axpy_dot size");
  if (nv > kBcgsFusedMax || !bcgs_fits(n, KB)) {
    bmaxpy(V, ldv, nv, h, W, n, KB, s);
    bmdot(V, ldv, nv, W, n, KB, part, out, s);
    return;
  }
  const int64_t G = bcgs_blocks(n, KB);
  switch ((nv + 7) / 8) {
#define FPC_CASE(B)                                                          \
  case B / 8:                                                                \
    if constexpr (B <= kBcgsFusedMax)                                        \
      k_bcgs_axpy_dot<B><<<(unsigned)G, BT, 0, s>>>(V, ldv, nv, h, W, n, KB, \
                                                   part);                   \
    break;
    FPC_BCGS_BUCKETS(FPC_CASE)
#undef FPC_CASE
  }
  FPC_LAUNCH_CHECK();
  k_bmdot_reduce<<<nv, BT, 0, s>>>(part, (int)G, KB, out);
  FPC_LAUNCH_CHECK();
}

void bcgs_axpy_norm(const double* V, int64_t ldv, int nv, const double* h,
                    double* W, int64_t n, int KB, double* part, double* out,
                    hipStream_t s) {
  if (nv < 1 || nv > kMaxKrylov || KB < 1 || KB > 32)
    throw Error(FPC_ERR_ARG, "bcgs_axpy_norm size");
  const int64_t G = bcgs_blocks(n, KB);
  k_bcgs_axpy_norm<<<(unsigned)G, BT, 0, s>>>(V, ldv, nv, h, W, n, KB, part);
  FPC_LAUNCH_CHECK();
  k_bmdot_reduce<<<1, BT, 0, s>>>(part, (int)G, KB, out);
  FPC_LAUNCH_CHECK();
}

void bmaxpy(const double* V, int64_t ldv, int nv, const double* h, double* W,
            int64_t n, int KB, hipStream_t s) {
  if (nv <= 0 || !n) return;
  if (nv > kMaxKrylov || KB > 32) throw Error(FPC_ERR_ARG, "bmaxpy size");
  unsigned g = grid_for(n * KB, BT);
  if (g > 16384) g = 16384;
  k_bmaxpy<<<g, BT, 0, s>>>(V, ldv, nv, h, W, n, KB);
  FPC_LAUNCH_CHECK();
}

// Largest vector count of one batched delayed dot launch (two sums per
// vector in registers).
constexpr int kBdcgsChunk = 32;

bool bdcgs_supported(int64_t n, int KB) { return n * KB < (int64_t(1) << 29); }

void bdcgs_dot(const double* V, int64_t ldv, int nv, const double* U,
               const double* W, int64_t n, int KB, double* part, double* D,
               hipStream_t s) {
  if (nv < 1 || nv > kMaxKrylov || KB < 1 || KB > 32 || !bdcgs_supported(n, KB))
    throw Error(FPC_ERR_ARG, "bdcgs_dot size");
  const int64_t G = bcgs_blocks(n, KB);
  for (int i0 = 0; i0 < nv; i0 += kBdcgsChunk) {
    const int cnt = std::min(kBdcgsChunk, nv - i0);
    const bool extra = i0 == 0;
    switch ((cnt + 7) / 8) {
#define FPC_CASE(B)                                                          \
  case B / 8:                                                                \
    if constexpr (B <= kBdcgsChunk) {                                        \
      if (W)                                                                 \
        k_bdcgs_dot<B, true><<<(unsigned)G, BT, 0, s>>>(                     \
            V, ldv, i0, cnt, nv, U, W, n, KB, extra, part);                  \
      else                                                                   \
        k_bdcgs_dot<B, false><<<(unsigned)G, BT, 0, s>>>(                    \
            V, ldv, i0, cnt, nv, U, W, n, KB, extra, part);                  \
    }                                                                        \
    break;
      FPC_BCGS_BUCKETS(FPC_CASE)
#undef FPC_CASE
    }
    FPC_LAUNCH_CHECK();
  }
  k_bmdot_reduce<<<W ? 2 * nv + 1 : nv, BT, 0, s>>>(part, (int)G, KB, D);
  FPC_LAUNCH_CHECK();
}

void bdcgs_finish(const double* D, int nv, bool fresh, const int* needfin,
                  double* H, int m, double* cs, double* sn, double* g,
                  double* P, double* rho, double* ww, double* sc, int* pf,
                  const int* active, int KB, hipStream_t s) {
  if (nv < 1 || nv > kMaxKrylov || KB < 1 || KB > 64)
    throw Error(FPC_ERR_ARG, "bdcgs_finish size");
  k_bdcgs_finish<<<1, 64, 0, s>>>(D, nv, fresh ? 1 : 0, needfin, H, m, cs, sn,
                                  g, P, rho, ww, sc, pf, active, KB);
  FPC_LAUNCH_CHECK();
}

void bdcgs_update(double* V, int64_t ldv, int j, const double* D,
                  const double* P, const double* rho, const double* W,
                  int64_t n, int KB, double* part, hipStream_t s) {
  if (j < 0 || j + 1 > kMaxKrylov || KB < 1 || KB > 32 || !bdcgs_supported(n, KB))
    throw Error(FPC_ERR_ARG, "bdcgs_update size");
  const int64_t G = bcgs_blocks(n, KB);
  switch ((std::max(j, 1) + 7) / 8) {
#define FPC_CASE(B)                                                          \
  case B / 8:                                                                \
    k_bdcgs_update<B><<<(unsigned)G, BT, 0, s>>>(V, ldv, j, D, P, rho, W, n, \
                                                 KB, part);                  \
    break;
    FPC_BCGS_BUCKETS(FPC_CASE)
#undef FPC_CASE
  }
  FPC_LAUNCH_CHECK();
}

void bdcgs_peek(const double* part, int64_t n, double* H, int m, double* cs,
                double* sn, double* g, const double* P, int j,
                const double* ww, double* sc, int* pf, const int* active,
                int KB, hipStream_t s) {
  k_bdcgs_peek<<<1, BT, 0, s>>>(part, (int)bcgs_blocks(n, KB), H, m, cs, sn,
                                g, P, j, ww, sc, pf, active, KB);
  FPC_LAUNCH_CHECK();
}

void bscale(const double* x, const double* scal, double* y, int64_t n, int KB,
            hipStream_t s) {
  k_bscale<<<grid_for(n * KB, 256), 256, 0, s>>>(x, scal, y, n, KB);
  FPC_LAUNCH_CHECK();
}

void bsub(const double* a, double* b, int64_t n, hipStream_t s) {
  k_bsub<<<grid_for(n, 256), 256, 0, s>>>(a, b, n);
  FPC_LAUNCH_CHECK();
}

void bgmres_step(double* H, double* cs, double* sn, double* g,
                 const double* h1, const double* h2, const double* nrm2,
                 const double* nrm0, int j, int m, int KB, const int* active,
                 double* scal, double* est, int* brk, hipStream_t s) {
  k_bgmres_step<<<1, 64, 0, s>>>(H, cs, sn, g, h1, h2, nrm2, nrm0, j, m, KB,
                                 active, scal, est, brk);
  FPC_LAUNCH_CHECK();
}

void bgmres_init(double* g, int m, int KB, const double* beta2,
                 const int* active, double* scal, hipStream_t s) {
  k_bgmres_init<<<1, 64, 0, s>>>(g, m, KB, beta2, active, scal);
  FPC_LAUNCH_CHECK();
}

void btrisolve(const double* H, const double* g, double* y, const int* kc,
               int m, int KB, hipStream_t s) {
  k_btrisolve<<<1, 64, 0, s>>>(H, g, y, kc, m, KB);
  FPC_LAUNCH_CHECK();
}

}  // namespace fpc
