// Setup kernels of the block preconditioner and of the smoothed-aggregation
// hierarchy: face-block inverses (H~ = Bdiag(H,3)), diagonal scaling,
// distance-2 MIS aggregation, tentative prolongator (per-aggregate QR of the
// rigid-body modes), prolongator smoothing, coarse dummy dofs, power-iteration
// start vectors and the blocked Gauss-Jordan inverse of dense matrices.
#include <type_traits>

#include "fpc_internal.hpp"

namespace fpc {

namespace {

constexpr int IDX_BITS = 28;
constexpr int64_t IDX_MASK = (int64_t(1) << IDX_BITS) - 1;

// ------------------------------------------------------------- H~^{-1}
__device__ inline double csr_get(const int64_t* rp, const int32_t* col,
                                 const double* val, int64_t row, int32_t c) {
  int64_t lo = rp[row], hi = rp[row + 1];
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (col[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  return (lo < rp[row + 1] && col[lo] == c) ? val[lo] : 0.0;
}

__global__ void k_hinv(const int64_t* rp, const int32_t* col,
                       const double* val, int64_t n_p, double* hinv,
                       int* flags) {
  int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= n_p) return;
  double a[9];
  double amax = 0.0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      a[r * 3 + c] = csr_get(rp, col, val, 3 * K + r, (int32_t)(3 * K + c));
      amax = fmax(amax, fabs(a[r * 3 + c]));
    }
  double c00 = a[4] * a[8] - a[5] * a[7];
  double c01 = a[5] * a[6] - a[3] * a[8];
  double c02 = a[3] * a[7] - a[4] * a[6];
  double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  if (!(fabs(det) > 1e-14 * amax * amax * amax) || !isfinite(det)) {
    atomicOr(&flags[FLAG_SINGULAR], 1);
    det = 1.0;
  }
  double* o = hinv + K * 9;
  o[0] = c00 / det;
  o[3] = c01 / det;
  o[6] = c02 / det;
  o[1] = (a[2] * a[7] - a[1] * a[8]) / det;
  o[4] = (a[0] * a[8] - a[2] * a[6]) / det;
  o[7] = (a[1] * a[6] - a[0] * a[7]) / det;
  o[2] = (a[1] * a[5] - a[2] * a[4]) / det;
  o[5] = (a[2] * a[3] - a[0] * a[5]) / det;
  o[8] = (a[0] * a[4] - a[1] * a[3]) / det;
}

__global__ void k_row_scale3(const int64_t* rp, double* val, int64_t nbr,
                             const double* blocks) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbr) return;
  const double* h = blocks + i * 9;
  for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
    double* v = val + e * 9;
    double t[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        t[r * 3 + c] = h[r * 3 + 0] * v[0 * 3 + c] + h[r * 3 + 1] * v[1 * 3 + c] +
                       h[r * 3 + 2] * v[2 * 3 + c];
    for (int q = 0; q < 9; ++q) v[q] = t[q];
  }
}

__global__ void k_dinv(const int64_t* rp, const int32_t* col,
                       const double* val, int64_t nbr, int br, int bc,
                       double* dinv, int* flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbr) return;
  int64_t e = -1;
  for (int64_t q = rp[i]; q < rp[i + 1]; ++q)
    if (col[q] == i) {
      e = q;
      break;
    }
  for (int r = 0; r < br; ++r) {
    double d = (e >= 0) ? val[e * br * bc + r * bc + r] : 0.0;
    if (!(d != 0.0) || !isfinite(d)) {
      atomicOr(&flags[FLAG_SINGULAR], 1);
      d = 1.0;
    }
    dinv[i * br + r] = 1.0 / d;
  }
}

// ------------------------------------------------------------- aggregation
__global__ void k_agg_init(const int64_t* rp, const int32_t* col, int64_t n,
                           int64_t* prio, int32_t* state, uint8_t* iso) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool has_off = false;
  for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
    if (col[e] != i) {
      has_off = true;
      break;
    }
  iso[i] = has_off ? 0 : 1;
  state[i] = has_off ? 1 : 0;
  prio[i] = ((int64_t)lowbias32((uint32_t)i) << IDX_BITS) | i;
}

__global__ void k_key(const int32_t* state, const int64_t* prio, int64_t n,
                      int64_t* key) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = ((int64_t)state[i] << 61) | prio[i];
}

// out[i] = max(in[i], max over the block row's columns)
// (four lanes per row, each taking every fourth neighbour, then a shuffle
// max: more gathers in flight than one lane per row)
__global__ void k_max_closed(const int64_t* rp, const int32_t* col,
                             int64_t n, const int64_t* in, int64_t* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t >> 2;
  const int q = (int)(t & 3);
  int64_t m = INT64_MIN;
  if (i < n) {
    if (q == 0) m = in[i];
    for (int64_t e = rp[i] + q; e < rp[i + 1]; e += 4) m = max(m, in[col[e]]);
  }
  m = max(m, (int64_t)__shfl_xor((long long)m, 1, 64));
  m = max(m, (int64_t)__shfl_xor((long long)m, 2, 64));
  if (i < n && q == 0) out[i] = m;
}

__global__ void k_mis_update(int32_t* state, const int64_t* key,
                             const int64_t* m2, int64_t n, int* undecided) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (state[i] != 1) return;
  if (m2[i] == key[i]) state[i] = 2;
  else if ((m2[i] >> 61) == 2) state[i] = 0;
  else atomicAdd(undecided, 1);
}

__global__ void k_is_root(const int32_t* state, int64_t n, int64_t* flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = state[i] == 2 ? 1 : 0;
}

__global__ void k_root_ids(const int32_t* state, const int64_t* scan,
                           int64_t n, int32_t* agg, int32_t* roots,
                           const int64_t* prio, int64_t* rk) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (state[i] == 2) {
    int32_t a = (int32_t)scan[i];
    agg[i] = a;
    roots[a] = (int32_t)i;
    rk[i] = prio[i];
  } else {
    agg[i] = -1;
    rk[i] = -1;
  }
}

__global__ void k_join(const uint8_t* iso, const int64_t* m, int64_t n,
                       int32_t* agg, int* remaining) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (iso[i] || agg[i] >= 0) return;
  if (m[i] >= 0) {
    int64_t root = m[i] & IDX_MASK;
    agg[i] = agg[root];
  } else {
    atomicAdd(remaining, 1);
  }
}

__global__ void k_rk2(const int32_t* agg, const int32_t* roots,
                      const int64_t* prio, int64_t n, int64_t* rk) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  rk[i] = agg[i] >= 0 ? prio[roots[agg[i]]] : -1;
}

// ------------------------------------------------------------- near-nullspace
__global__ void k_bbox_partial(const double* X, int64_t n, double* part) {
  __shared__ double sh[6][256];
  double mn[3] = {INFINITY, INFINITY, INFINITY};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    for (int d = 0; d < 3; ++d) {
      mn[d] = fmin(mn[d], X[i * 3 + d]);
      mx[d] = fmax(mx[d], X[i * 3 + d]);
    }
  for (int d = 0; d < 3; ++d) {
    sh[d][threadIdx.x] = mn[d];
    sh[3 + d][threadIdx.x] = mx[d];
  }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + s]);
        sh[3 + d][threadIdx.x] =
            fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int d = 0; d < 6; ++d) part[blockIdx.x * 6 + d] = sh[d][0];
}

__global__ void k_bbox_final(const double* part, int np, double* ctr) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int d = 0; d < 3; ++d) {
    double mn = INFINITY, mx = -INFINITY;
    for (int b = 0; b < np; ++b) {
      mn = fmin(mn, part[b * 6 + d]);
      mx = fmax(mx, part[b * 6 + 3 + d]);
    }
    ctr[d] = 0.5 * (mn + mx);
  }
}

__global__ void k_rigid(const double* X, const double* ctr, int64_t n, int nb,
                        double* B) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double* b = B + i * 3 * nb;
  for (int q = 0; q < 3 * nb; ++q) b[q] = 0.0;
  for (int c = 0; c < 3; ++c) b[c * nb + c] = 1.0;
  if (nb == 6) {
    double y0 = X[i * 3 + 0] - ctr[0];
    double y1 = X[i * 3 + 1] - ctr[1];
    double y2 = X[i * 3 + 2] - ctr[2];
    // rotation about x: (0, -y_z, y_y); about y: (y_z, 0, -y_x);
    // about z: (-y_y, y_x, 0)
    b[1 * nb + 3] = -y2;
    b[2 * nb + 3] = y1;
    b[0 * nb + 4] = y2;
    b[2 * nb + 4] = -y0;
    b[0 * nb + 5] = -y1;
    b[1 * nb + 5] = y0;
  }
}

// ------------------------------------------------------------- tentative P
__global__ void k_agg_count(const int32_t* agg, int64_t n,
                            unsigned long long* cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (agg[i] >= 0) atomicAdd(&cnt[agg[i]], 1ull);
}

__global__ void k_agg_fill(const int32_t* agg, int64_t n,
                           unsigned long long* cursor, int32_t* members) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (agg[i] >= 0) members[atomicAdd(&cursor[agg[i]], 1ull)] = (int32_t)i;
}

// Rows (members x block size) an aggregate may have for k_tentative_w.
constexpr int TENT_ROWS = 2048;

// Insertion sort of the members of the aggregates with more than min_rows
// rows (the others are sorted inside k_tentative_w).
__global__ void k_agg_sort(const int64_t* off, int64_t n_agg, int bs,
                           int64_t min_rows, int32_t* members) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_agg) return;
  if ((off[a + 1] - off[a]) * bs <= min_rows) return;
  for (int64_t e = off[a] + 1; e < off[a + 1]; ++e) {
    int32_t v = members[e];
    int64_t f = e - 1;
    while (f >= off[a] && members[f] > v) {
      members[f + 1] = members[f];
      --f;
    }
    members[f + 1] = v;
  }
}

// Per aggregate: thin QR of the stacked near-nullspace rows of its members
// by modified Gram-Schmidt applied twice; columns whose remaining norm is
// <= drop_tol * (largest column norm) are dropped.  Q is written over the
// rows of ptent (kept columns first, the rest zero), R into Bc.
// (Thread per aggregate; used for the aggregates with more than min_rows
// rows.)
__global__ void k_tentative(const int64_t* off, const int32_t* members,
                            int64_t n_agg, int bs, int nb, const double* B,
                            double drop_tol, double* ptent, double* Bc,
                            int32_t* rank, int64_t min_rows) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_agg) return;
  const int64_t m0 = off[a], m1 = off[a + 1];
  if ((m1 - m0) * bs <= min_rows) return;
  double R[36];
  for (int q = 0; q < 36; ++q) R[q] = 0.0;
  double scale = 0.0;
  for (int j = 0; j < nb; ++j) {
    double s = 0.0;
    for (int64_t e = m0; e < m1; ++e) {
      const double* b = B + (int64_t)members[e] * bs * nb;
      for (int c = 0; c < bs; ++c) s += b[c * nb + j] * b[c * nb + j];
    }
    scale = fmax(scale, sqrt(s));
  }
  int kc = 0;
  for (int j = 0; j < nb; ++j) {
    for (int64_t e = m0; e < m1; ++e) {
      const int64_t node = members[e];
      for (int c = 0; c < bs; ++c)
        ptent[(node * bs + c) * nb + kc] = B[(node * bs + c) * nb + j];
    }
    for (int pass = 0; pass < 2; ++pass)
      for (int k = 0; k < kc; ++k) {
        double d = 0.0;
        for (int64_t e = m0; e < m1; ++e) {
          const double* p = ptent + (int64_t)members[e] * bs * nb;
          for (int c = 0; c < bs; ++c) d += p[c * nb + k] * p[c * nb + kc];
        }
        R[k * 6 + j] += d;
        for (int64_t e = m0; e < m1; ++e) {
          double* p = ptent + (int64_t)members[e] * bs * nb;
          for (int c = 0; c < bs; ++c) p[c * nb + kc] -= d * p[c * nb + k];
        }
      }
    double nv = 0.0;
    for (int64_t e = m0; e < m1; ++e) {
      const double* p = ptent + (int64_t)members[e] * bs * nb;
      for (int c = 0; c < bs; ++c) nv += p[c * nb + kc] * p[c * nb + kc];
    }
    nv = sqrt(nv);
    if (nv > drop_tol * scale) {
      R[kc * 6 + j] = nv;
      for (int64_t e = m0; e < m1; ++e) {
        double* p = ptent + (int64_t)members[e] * bs * nb;
        for (int c = 0; c < bs; ++c) p[c * nb + kc] = p[c * nb + kc] / nv;
      }
      ++kc;
    }
  }
  for (int64_t e = m0; e < m1; ++e) {
    double* p = ptent + (int64_t)members[e] * bs * nb;
    for (int c = 0; c < bs; ++c)
      for (int k = kc; k < nb; ++k) p[c * nb + k] = 0.0;
  }
  rank[a] = kc;
  double* o = Bc + a * nb * nb;
  for (int k = 0; k < nb; ++k)
    for (int j = 0; j < nb; ++j) o[k * nb + j] = (k < kc) ? R[k * 6 + j] : 0.0;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the WPA waves of one aggregate group, in a fixed order, so every
// thread of the group gets the same value.
template <int WPA>
__device__ inline double group_sum(double v, double* red) {
  v = wave_sum(v);
  if constexpr (WPA == 1) {
    return v;
  } else {
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int i = 1; i < WPA; ++i) r += red[i];
    __syncthreads();
    return r;
  }
}

// The same QR as k_tentative, with WPA waves per aggregate and T rows per
// thread, for aggregates with lo < rows <= 64 * WPA * T (a 256-thread block
// holds 4 / WPA aggregates).  Thread g of the group holds rows g, g + 64 WPA,
// ... of the stacked block; the members are first put in ascending order in
// LDS (rank sort).  Dot products are butterfly sums over the wave, then over
// the group's waves in a fixed order, identical in every thread, so all take
// the same keep/drop decision.
template <int WPA, int T>
__global__ __launch_bounds__(256) void k_tentative_w(
    const int64_t* off, const int32_t* members, int64_t n_agg, int bs, int nb,
    const double* B, double drop_tol, double* ptent, double* Bc,
    int32_t* rank, int64_t lo) {
  constexpr int GS = 64 * WPA;    // threads per aggregate
  constexpr int CAP = GS * T;     // rows per aggregate
  __shared__ int32_t smem[4 / WPA][CAP];
  __shared__ double red[4];
  const int g = threadIdx.x % GS;
  const int grp = threadIdx.x / GS;
  const int64_t a = (int64_t)blockIdx.x * (4 / WPA) + grp;
  const int64_t m0 = a < n_agg ? off[a] : 0;
  const int64_t len = a < n_agg ? off[a + 1] - m0 : 0;
  const bool valid = a < n_agg && len * bs > lo && len * bs <= CAP;
  // groups without work keep m = 0 and take part in the barriers only
  const int m = valid ? (int)len : 0;
  const int M = m * bs;
  int32_t* sm = smem[grp];
  int32_t mine[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int e = g + GS * t;
    mine[t] = e < m ? members[m0 + e] : 0;
    if (e < m) sm[e] = mine[t];
  }
  __syncthreads();
  int32_t sorted_pos[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    int r = 0;
    if (g + GS * t < m)
      for (int f = 0; f < m; ++f) r += sm[f] < mine[t];
    sorted_pos[t] = r;
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < T; ++t)
    if (g + GS * t < m) sm[sorted_pos[t]] = mine[t];
  __syncthreads();
  // past the last barrier shared by groups (with WPA = 4 the block is one
  // aggregate, so valid is uniform over the block)
  if (!valid) return;
  double Q[T][6];
  int64_t rowoff[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int rho = g + GS * t;
    const bool in = rho < M;
    const int64_t node = in ? sm[rho / bs] : 0;
    rowoff[t] = in ? (node * bs + rho % bs) * nb : -1;
#pragma unroll
    for (int j = 0; j < 6; ++j) Q[t][j] = 0.0;
  }
  double* o = Bc + a * nb * nb;
  if (g == 0)
    for (int q = 0; q < nb * nb; ++q) o[q] = 0.0;
  double scale = 0.0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    if (j >= nb) break;
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const double x = rowoff[t] >= 0 ? B[rowoff[t] + j] : 0.0;
      v += x * x;
    }
    scale = fmax(scale, sqrt(group_sum<WPA>(v, red)));
  }
  int kc = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    if (j >= nb) break;
    double v[T];
#pragma unroll
    for (int t = 0; t < T; ++t) v[t] = rowoff[t] >= 0 ? B[rowoff[t] + j] : 0.0;
    double rj[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int pass = 0; pass < 2; ++pass)
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        if (k >= kc) break;
        double d = 0.0;
#pragma unroll
        for (int t = 0; t < T; ++t) d += Q[t][k] * v[t];
        d = group_sum<WPA>(d, red);
        rj[k] += d;
#pragma unroll
        for (int t = 0; t < T; ++t) v[t] -= d * Q[t][k];
      }
    double nv = 0.0;
#pragma unroll
    for (int t = 0; t < T; ++t) nv += v[t] * v[t];
    nv = sqrt(group_sum<WPA>(nv, red));
    const bool keep = nv > drop_tol * scale;
    if (g == 0) {
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (k < kc) o[k * nb + j] = rj[k];
      if (keep) o[kc * nb + j] = nv;
    }
    if (keep) {
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (k == kc)
#pragma unroll
          for (int t = 0; t < T; ++t) Q[t][k] = v[t] / nv;
      ++kc;
    }
  }
#pragma unroll
  for (int t = 0; t < T; ++t)
    if (rowoff[t] >= 0)
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (k < nb) ptent[rowoff[t] + k] = Q[t][k];
  if (g == 0) rank[a] = kc;
}

__global__ void k_ptent_count(const int32_t* agg, int64_t n, int64_t* cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cnt[i] = agg[i] >= 0 ? 1 : 0;
}

__global__ void k_ptent_fill(const int32_t* agg, const int64_t* rp, int64_t n,
                             int B, const double* ptent, int32_t* col,
                             double* val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (agg[i] < 0) return;
  int64_t e = rp[i];
  col[e] = agg[i];
  for (int q = 0; q < B; ++q) val[e * B + q] = ptent[i * B + q];
}

// val <- -(omega * dinv[row scalar]) * val, one wavefront per block row: a
// block row's values are contiguous, so the lanes stride them directly.
__global__ __launch_bounds__(256) void k_neg_row_scale(const int64_t* rp,
                                                       double* val, int64_t nbr,
                                                       int br, int bc,
                                                       const double* dinv,
                                                       double omega) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nbr) return;
  const int B = br * bc;
  const int64_t v0 = rp[i] * B, v1 = rp[i + 1] * B;
  for (int64_t v = v0 + lane; v < v1; v += 64) {
    const int r = (int)((v - v0) % B) / bc;
    const double t = omega * dinv[i * br + r];
    val[v] = -(t * val[v]);
  }
}

__global__ void k_dummy_diag(const int64_t* rp, const int32_t* col,
                             double* val, int64_t nbr, int nb,
                             const int32_t* rank) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nbr) return;
  for (int64_t e = rp[a]; e < rp[a + 1]; ++e)
    if (col[e] == a) {
      for (int k = rank[a]; k < nb; ++k) val[e * nb * nb + k * nb + k] = 1.0;
      return;
    }
}

__global__ void k_power_start(int64_t n_nodes, int bs, int stride,
                              const int32_t* node_rank, double* x) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_nodes * bs) return;
  int64_t node = i / bs;
  int c = (int)(i % bs);
  if (node_rank && c >= node_rank[node]) {
    x[i] = 0.0;
    return;
  }
  uint32_t h = lowbias32((uint32_t)(stride * node + c));
  x[i] = (double)h / 4294967296.0 - 0.5;
}

// One workgroup per block row: its threads stride over the row's values
// (the coarsest operator's rows hold hundreds of blocks).
__global__ __launch_bounds__(256) void k_dense_from_bsr(
    const int64_t* rp, const int32_t* col, const double* val, int64_t nbr,
    int br, int bc, int64_t npad, double* D) {
  const int64_t i = blockIdx.x;
  if (i >= nbr) return;
  const int bs = br * bc;
  const int64_t e0 = rp[i], n = (rp[i + 1] - e0) * bs;
  for (int64_t idx = threadIdx.x; idx < n; idx += 256) {
    const int64_t e = e0 + idx / bs;
    const int q = (int)(idx % bs), r = q / bc, c = q % bc;
    D[(i * br + r) * npad + (int64_t)col[e] * bc + c] = val[e * bs + q];
  }
}

__global__ void k_pad_identity(double* D, int64_t n, int64_t npad) {
  int64_t i = n + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < npad) D[i * npad + i] = 1.0;
}

// ------------------------------------------------------------- dense GJ
// Dense inverse of the coarsest Galerkin operator in place: Gauss-Jordan
// with partial pivoting in 256-wide panels.  Each panel's pivot rows come
// from an LU with partial pivoting of the panel's columns and are exchanged
// first; the diagonal block is then inverted without further exchanges by
// the 64-wide tile kernels, and the row panel, trailing update and column
// panel are FP64 MFMA products (k_gemm_f64).  `ld` is the row pitch, `n` the
// order.
constexpr int GT = 64;  // tile

// Gauss-Jordan inverse of the diagonal tile, in place.  Thread (tr, tc)
// keeps rows 4tr..4tr+3 x columns 4tc..4tc+3 in registers; at step k the
// owners of row k and of column k publish them in LDS (two buffers, so one
// barrier per step) and every thread updates its 16 entries.
__global__ __launch_bounds__(256) void k_gj_diag(double* D, int64_t ld,
                                                 int64_t kb, int spd,
                                                 int* flags) {
  __shared__ double rowb[2][GT];
  __shared__ double colb[2][GT];
  const int tid = threadIdx.x;
  const int tr = tid >> 4, tc = tid & 15;
  const int64_t o = kb * GT;
  double a[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      a[i][j] = D[(o + 4 * tr + i) * ld + o + 4 * tc + j];
  // one elimination step; the pivot's position inside the owners' 4 x 4
  // blocks (KR) is a compile-time constant, so no register is indexed at run
  // time
  auto step = [&](const int k, auto kr_c) {
    constexpr int kr = decltype(kr_c)::value;
    const int buf = k & 1;
    const int kq = k >> 2;
    // owners publish row k and column k
    if (tr == kq) {
#pragma unroll
      for (int j = 0; j < 4; ++j) rowb[buf][4 * tc + j] = a[kr][j];
    }
    if (tc == kq) {
#pragma unroll
      for (int i = 0; i < 4; ++i) colb[buf][4 * tr + i] = a[i][kr];
    }
    __syncthreads();
    // all reads of the step issued together
    double p = rowb[buf][k];
    double rv[4], pc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) rv[j] = rowb[buf][4 * tc + j];
#pragma unroll
    for (int i = 0; i < 4; ++i) pc[i] = colb[buf][4 * tr + i];
    const bool bad = spd ? !(p > 0.0) : !(fabs(p) > 0.0);
    if (bad || !isfinite(p)) {
      if (tid == 0) atomicOr(&flags[spd ? FLAG_NOT_SPD : FLAG_SINGULAR], 1);
      p = 1.0;
    }
    const double ip = 1.0 / p;
    double pr[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) pr[j] = (4 * tc + j == k) ? ip : rv[j] * ip;
    // a_rc -= a_rk a_kc / p everywhere, then the owners overwrite column k
    // (-a_rk / p) and row k (a_kc / p, and 1 / p on the diagonal)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) a[i][j] -= pc[i] * pr[j];
    if (tc == kq) {
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i][kr] = -pc[i] * ip;
    }
    if (tr == kq) {
#pragma unroll
      for (int j = 0; j < 4; ++j) a[kr][j] = pr[j];
    }
  };
  for (int k0 = 0; k0 < GT; k0 += 4) {
    step(k0, std::integral_constant<int, 0>{});
    step(k0 + 1, std::integral_constant<int, 1>{});
    step(k0 + 2, std::integral_constant<int, 2>{});
    step(k0 + 3, std::integral_constant<int, 3>{});
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      D[(o + 4 * tr + i) * ld + o + 4 * tc + j] = a[i][j];
}

// acc = X(xi, xj) * Y(yi, yj) for 64x64 tiles (tile coordinates).
__device__ inline void tile_gemm(const double* D, int64_t ld, int64_t xi,
                                 int64_t xj, int64_t yi, int64_t yj,
                                 double (*sa)[GT + 1], double (*sb)[GT + 1],
                                 double acc[4][4]) {
  const int tid = threadIdx.x;
  {
    // all 32 loads of a thread in flight before the LDS stores
    const int c = tid & (GT - 1), r0 = tid >> 6;
    double ra[16], rb[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t r = r0 + 4 * u;
      ra[u] = D[(xi * GT + r) * ld + xj * GT + c];
      rb[u] = D[(yi * GT + r) * ld + yj * GT + c];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      sa[r0 + 4 * u][c] = ra[u];
      sb[r0 + 4 * u][c] = rb[u];
    }
  }
  __syncthreads();
  const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k = 0; k < GT; ++k) {
    double x[4], y[4];
    for (int i = 0; i < 4; ++i) x[i] = sa[tr + i][k];
    for (int j = 0; j < 4; ++j) y[j] = sb[k][tc + j];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) acc[i][j] += x[i] * y[j];
  }
}

// row panel: A[kb, j] <- Dinv * A[kb, j], j != kb
__global__ __launch_bounds__(256) void k_gj_rowpanel(double* D, int64_t ld,
                                                     int64_t kb) {
  __shared__ double sa[GT][GT + 1];
  __shared__ double sb[GT][GT + 1];
  int64_t j = blockIdx.x;
  if (j >= kb) ++j;
  double acc[4][4];
  tile_gemm(D, ld, kb, kb, kb, j, sa, sb, acc);
  __syncthreads();
  const int tr = (threadIdx.x / 16) * 4, tc = (threadIdx.x % 16) * 4;
  for (int i = 0; i < 4; ++i)
    for (int jj = 0; jj < 4; ++jj)
      D[(kb * GT + tr + i) * ld + j * GT + tc + jj] = acc[i][jj];
}

// trailing update: A[i, j] -= A[i, kb] A[kb, j], i != kb, j != kb
__global__ __launch_bounds__(256) void k_gj_update(double* D, int64_t ld,
                                                   int64_t kb, int64_t nt) {
  __shared__ double sa[GT][GT + 1];
  __shared__ double sb[GT][GT + 1];
  int64_t t = blockIdx.x;
  int64_t i = t / (nt - 1), j = t % (nt - 1);
  if (i >= kb) ++i;
  if (j >= kb) ++j;
  double acc[4][4];
  tile_gemm(D, ld, i, kb, kb, j, sa, sb, acc);
  const int tr = (threadIdx.x / 16) * 4, tc = (threadIdx.x % 16) * 4;
  // the 16 old values are loaded together, then updated and stored
  double old[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      old[r][c] = D[(i * GT + tr + r) * ld + j * GT + tc + c];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      D[(i * GT + tr + r) * ld + j * GT + tc + c] = old[r][c] - acc[r][c];
}

// column panel: A[i, kb] <- -A[i, kb] * Dinv, i != kb
__global__ __launch_bounds__(256) void k_gj_colpanel(double* D, int64_t ld,
                                                     int64_t kb) {
  __shared__ double sa[GT][GT + 1];
  __shared__ double sb[GT][GT + 1];
  int64_t i = blockIdx.x;
  if (i >= kb) ++i;
  double acc[4][4];
  tile_gemm(D, ld, i, kb, kb, kb, sa, sb, acc);
  __syncthreads();
  const int tr = (threadIdx.x / 16) * 4, tc = (threadIdx.x % 16) * 4;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c)
      D[(i * GT + tr + r) * ld + kb * GT + tc + c] = -acc[r][c];
}

// Logical index l -> physical index: the range [at, at + len) is skipped.
// Logical -> stored row (or column) index of a GEMM operand: either the
// identity with the range [at, at + len) skipped, or (tiles != null) the
// 64-row tiles listed in `tiles`, in order.
struct SkipMap {
  int64_t at, len;
  const int32_t* tiles = nullptr;
  __device__ int64_t operator()(int64_t l) const {
    if (tiles) return (int64_t)tiles[l >> 6] * 64 + (l & 63);
    return l < at ? l : l + len;
  }
};

// C[rm(i), cm(j)] = alpha * sum_k A[rm(i), k] B[k, cm(j)] + beta * C[..]
// (row-major, pitches lda / ldb / ldc).  128 x 128 output tile per
// workgroup, 64 x 64 per wavefront as 4 x 4 tiles of v_mfma_f64_16x16x4f64,
// K in chunks of 16 through LDS with the next chunk's loads in flight during
// the products.  Operand layout of that instruction: lane l holds A[l%16]
// [l/16] and B[l/16][l%16]; result register r of lane l is D[l/16 + 4r]
// [l%16].  Requires K and N multiples of 16 and skip offsets that are
// multiples of 8 (eight consecutive logical columns stay contiguous).
constexpr int GM_T = 128, GM_KC = 16, GM_LP = 16;

__global__ __launch_bounds__(256, 2) void k_gemm_f64(
    int64_t M, int64_t N, int K, double alpha, double beta,
    const double* __restrict__ A, int64_t lda, const double* __restrict__ B,
    int64_t ldb, double* __restrict__ C, int64_t ldc, SkipMap rm, SkipMap cm,
    int lower) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int AQ = GM_KC / 2, BQ = GM_KC * GM_T / 256;
  __shared__ double As[GM_KC][GM_T + GM_LP];
  __shared__ double Bs[GM_KC][GM_T + GM_LP];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t tiles_n = (N + GM_T - 1) / GM_T;
  const int64_t i0 = (int64_t)(blockIdx.x / tiles_n) * GM_T;
  const int64_t j0 = (int64_t)(blockIdx.x % tiles_n) * GM_T;
  // lower: only tiles reaching the lower triangle (i >= j) are computed
  if (lower && i0 + GM_T - 1 < j0) return;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  const int ar = tid >> 1, ak = (tid & 1) * AQ;
  const int bk = tid / (GM_T / BQ), bc = (tid % (GM_T / BQ)) * BQ;
  const bool aok = i0 + ar < M;
  const double* __restrict__ ap = A + (aok ? rm(i0 + ar) : 0) * lda + ak;
  const bool bok = j0 + bc < N;
  const double* __restrict__ bp = B + (int64_t)bk * ldb + (bok ? cm(j0 + bc) : 0);
  double av[AQ], bv[BQ];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < AQ; ++q) av[q] = aok ? ap[k0 + q] : 0.0;
#pragma unroll
    for (int q = 0; q < BQ; ++q) bv[q] = bok ? bp[(int64_t)k0 * ldb + q] : 0.0;
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += GM_KC) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < AQ; ++q) As[ak + q][ar] = av[q];
#pragma unroll
    for (int q = 0; q < BQ; ++q) Bs[bk][bc + q] = bv[q];
    __syncthreads();
    if (k0 + GM_KC < K) load(k0 + GM_KC);
#pragma unroll
    for (int kk = 0; kk < GM_KC; kk += 4) {
      double af[4], bf[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) af[a] = As[kk + (lane >> 4)][wm + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 4; ++b) bf[b] = Bs[kk + (lane >> 4)][wn + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t gi = i0 + wm + a * 16 + (lane >> 4) + 4 * r;
      if (gi >= M) continue;
      double* __restrict__ crow = C + rm(gi) * ldc;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t gj = j0 + wn + b * 16 + (lane & 15);
        if (gj < N) {
          double* c = crow + cm(gj);
          const double v = alpha * acc[a][b][r];
          *c = beta == 0.0 ? v : beta * *c + v;
        }
      }
    }
}

void gemm_f64(int64_t M, int64_t N, int K, double alpha, double beta,
              const double* A, int64_t lda, const double* B, int64_t ldb,
              double* C, int64_t ldc, SkipMap rm, SkipMap cm, hipStream_t s,
              int lower = 0) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  if (K % GM_KC || N % 16 || (rm.len && (rm.at % 8 || rm.len % 8)) ||
      (cm.len && (cm.at % 8 || cm.len % 8)))
    throw Error(FPC_ERR_ARG, "gemm_f64: shape not supported");
  const int64_t tiles = ((M + GM_T - 1) / GM_T) * ((N + GM_T - 1) / GM_T);
  k_gemm_f64<<<(unsigned)tiles, 256, 0, s>>>(M, N, K, alpha, beta, A, lda, B,
                                              ldb, C, ldc, rm, cm, lower);
  FPC_LAUNCH_CHECK();
}

// dst[c * ldd + r] = src[r * lds + c] for r < rows, c < cols (32 x 32 tiles)
void gj_inverse64(double* D, int64_t n, int64_t ld, int spd, int* flags,
                  hipStream_t s) {
  const int64_t nt = n / GT;
  for (int64_t kb = 0; kb < nt; ++kb) {
    k_gj_diag<<<1, 256, 0, s>>>(D, ld, kb, spd, flags);
    if (nt > 1) {
      k_gj_rowpanel<<<(unsigned)(nt - 1), 256, 0, s>>>(D, ld, kb);
      k_gj_update<<<(unsigned)((nt - 1) * (nt - 1)), 256, 0, s>>>(D, ld, kb,
                                                                  nt);
      k_gj_colpanel<<<(unsigned)(nt - 1), 256, 0, s>>>(D, ld, kb);
    }
    FPC_LAUNCH_CHECK();
  }
}

// ------------------------------------------------------------- fixed stress
constexpr int FS_KMAX = 64;

// entry (r, c) of a 3 x 3 block matrix with sorted block columns
__device__ inline double bsr3_get(const int64_t* rp, const int32_t* col,
                                  const double* val, int64_t r, int64_t c) {
  const int64_t br = r / 3, bc = c / 3;
  int64_t lo = rp[br], hi = rp[br + 1];
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (col[mid] < bc) lo = mid + 1;
    else hi = mid;
  }
  return (lo < rp[br + 1] && col[lo] == bc) ? val[lo * 9 + (r % 3) * 3 + c % 3]
                                             : 0.0;
}

// Algebraic fixed stress (eq. Ak, eq. FS_algebraic), one wavefront per face
// k: K = nz(Q1 column k) U nz(Q2 row k) (scalar dofs), S1^(k) = S1[K, K],
// [S_K]_k = Q2[k, K] S1^(k)^{-1} Q1[K, k]; faces with an empty Q2 row give 0.
// The dense solve is Gaussian elimination with partial pivoting in LDS.
__global__ __launch_bounds__(64) void k_fixed_stress(
    const int64_t* __restrict__ srp, const int32_t* __restrict__ scol,
    const double* __restrict__ sval, const int64_t* __restrict__ arp,
    const int32_t* __restrict__ acol, const double* __restrict__ aval,
    const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol,
    const double* __restrict__ bval, int64_t n_p, double* __restrict__ out,
    int* flags) {
  __shared__ double Sk[FS_KMAX][FS_KMAX + 1];
  __shared__ double q1[FS_KMAX], q2[FS_KMAX];
  __shared__ int32_t idx[FS_KMAX];
  __shared__ int nK, piv;
  const int64_t k = blockIdx.x;
  const int lane = threadIdx.x;
  if (k >= n_p) return;
  const int64_t b0 = brp[k], b1 = brp[k + 1];   // Q2 row k
  if (b0 == b1) {
    if (lane == 0) out[k] = 0.0;
    return;
  }
  if (lane == 0) {
    const int64_t a0 = arp[k], a1 = arp[k + 1];  // Q1^T row k = Q1 column k
    int n = 0;
    int64_t i = a0, j = b0;
    bool over = false;
    while (i < a1 || j < b1) {
      int32_t c;
      double v1 = 0.0, v2 = 0.0;
      if (j >= b1 || (i < a1 && acol[i] < bcol[j])) {
        c = acol[i];
        v1 = aval[i++];
      } else if (i >= a1 || bcol[j] < acol[i]) {
        c = bcol[j];
        v2 = bval[j++];
      } else {
        c = acol[i];
        v1 = aval[i++];
        v2 = bval[j++];
      }
      if (n == FS_KMAX) {
        over = true;
        break;
      }
      idx[n] = c;
      q1[n] = v1;
      q2[n] = v2;
      ++n;
    }
    nK = over ? -1 : n;
  }
  __syncthreads();
  const int n = nK;
  if (n < 0) {
    if (lane == 0) {
      atomicOr(&flags[FLAG_OVERFLOW], 1);
      out[k] = 0.0;
    }
    return;
  }
  for (int e = lane; e < n * n; e += 64) {
    const int r = e / n, c = e % n;
    Sk[r][c] = bsr3_get(srp, scol, sval, idx[r], idx[c]);
  }
  __syncthreads();
  for (int c = 0; c < n; ++c) {
    if (lane == 0) {
      int p = c;
      double best = fabs(Sk[c][c]);
      for (int r = c + 1; r < n; ++r)
        if (fabs(Sk[r][c]) > best) {
          best = fabs(Sk[r][c]);
          p = r;
        }
      piv = p;
      if (!(best > 0.0) || !isfinite(best)) atomicOr(&flags[FLAG_SINGULAR], 1);
    }
    __syncthreads();
    const int p = piv;
    if (p != c) {
      for (int j = lane; j < n; j += 64) {
        const double t = Sk[c][j];
        Sk[c][j] = Sk[p][j];
        Sk[p][j] = t;
      }
      if (lane == 0) {
        const double t = q1[c];
        q1[c] = q1[p];
        q1[p] = t;
      }
    }
    __syncthreads();
    const double d = Sk[c][c] != 0.0 ? Sk[c][c] : 1.0;
    for (int r = c + 1 + lane; r < n; r += 64) {
      const double f = Sk[r][c] / d;
      for (int j = c + 1; j < n; ++j) Sk[r][j] -= f * Sk[c][j];
      q1[r] -= f * q1[c];
    }
    __syncthreads();
  }
  if (lane == 0) {
    for (int r = n - 1; r >= 0; --r) {
      double t = q1[r];
      for (int j = r + 1; j < n; ++j) t -= Sk[r][j] * q1[j];
      q1[r] = t / (Sk[r][r] != 0.0 ? Sk[r][r] : 1.0);
    }
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += q2[i] * q1[i];
    out[k] = acc;
  }
}

// Block row i of a BSR with one-row blocks times alpha / M[i][i] (M a
// square CSR): -T~^{-1} Q2 with T~ = diag(T) for the t-p-u surrogate.
__global__ void k_row_scale_inv_diag(const int64_t* rp, double* val,
                                     int64_t nbr, int bc,
                                     const int64_t* mrp, const int32_t* mcol,
                                     const double* mval, double alpha,
                                     int* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbr) return;
  double d = csr_get(mrp, mcol, mval, i, (int32_t)i);
  if (!(d != 0.0) || !isfinite(d)) {
    atomicOr(&flags[FLAG_SINGULAR], 1);
    d = 1.0;
  }
  const double f = alpha / d;
  for (int64_t e = rp[i] * bc; e < rp[i + 1] * bc; ++e) val[e] *= f;
}

}  // namespace

void hinv_setup(const Csr& H, int64_t n_p, double* hinv, int* flags,
                hipStream_t s) {
  if (n_p == 0) return;
  k_hinv<<<grid_for(n_p, 128), 128, 0, s>>>(H.rowptr.p, H.col.p, H.val.p, n_p,
                                            hinv, flags);
  FPC_LAUNCH_CHECK();
}

void bsr_block_row_scale(Bsr& b, const double* blocks3x3, hipStream_t s) {
  if (b.br != 3 || b.bc != 3)
    throw Error(FPC_ERR_ARG, "row scale expects 3x3 blocks");
  if (b.nbr == 0) return;
  k_row_scale3<<<grid_for(b.nbr, 128), 128, 0, s>>>(b.rowptr.p, b.val.p,
                                                    b.nbr, blocks3x3);
  FPC_LAUNCH_CHECK();
}

void bsr_dinv(const Bsr& a, double* dinv, int* flags, hipStream_t s) {
  if (a.nbr == 0) return;
  k_dinv<<<grid_for(a.nbr, 128), 128, 0, s>>>(a.rowptr.p, a.col.p, a.val.p,
                                              a.nbr, a.br, a.bc, dinv, flags);
  FPC_LAUNCH_CHECK();
}

int64_t aggregate_mis2(const Bsr& a, int32_t* agg, DevBuf<int32_t>& roots,
                       hipStream_t s) {
  const int64_t n = a.nbr;
  if (n >= (int64_t(1) << IDX_BITS))
    throw Error(FPC_ERR_UNSUPPORTED, "too many nodes for aggregation keys");
  DevBuf<int64_t> prio(n), key(n), m1(n), m2(n);
  DevBuf<int32_t> state(n);
  DevBuf<uint8_t> iso(n);
  DevBuf<int> cnt(1);
  const unsigned g = grid_for(n, 256);
  const unsigned g4 = grid_for(4 * n, 256);  // k_max_closed: four lanes a row
  k_agg_init<<<g, 256, 0, s>>>(a.rowptr.p, a.col.p, n, prio.p, state.p, iso.p);
  FPC_LAUNCH_CHECK();
  // four rounds per check (a round after convergence changes nothing); the
  // count is that of the batch's last round
  for (int round = 0; round < 1000; round += 4) {
    for (int k = 0; k < 4; ++k) {
      if (k == 3) FPC_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int), s));
      k_key<<<g, 256, 0, s>>>(state.p, prio.p, n, key.p);
      k_max_closed<<<g4, 256, 0, s>>>(a.rowptr.p, a.col.p, n, key.p, m1.p);
      k_max_closed<<<g4, 256, 0, s>>>(a.rowptr.p, a.col.p, n, m1.p, m2.p);
      k_mis_update<<<g, 256, 0, s>>>(state.p, key.p, m2.p, n, cnt.p);
    }
    FPC_LAUNCH_CHECK();
    if (read_i32(cnt.p, s) == 0) break;
    if (round >= 996) throw Error(FPC_ERR_HIP, "MIS-2 did not terminate");
  }
  DevBuf<int64_t> flag(n), scan(n + 1);
  k_is_root<<<g, 256, 0, s>>>(state.p, n, flag.p);
  FPC_LAUNCH_CHECK();
  const int64_t n_agg = scan_counts_total(flag.p, scan.p, n, s);
  roots.alloc(std::max<int64_t>(n_agg, 1));
  k_root_ids<<<g, 256, 0, s>>>(state.p, scan.p, n, agg, roots.p, prio.p,
                               key.p);
  FPC_LAUNCH_CHECK();
  // phase 1: join the adjacent root of largest priority
  k_max_closed<<<g4, 256, 0, s>>>(a.rowptr.p, a.col.p, n, key.p, m1.p);
  FPC_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int), s));
  k_join<<<g, 256, 0, s>>>(iso.p, m1.p, n, agg, cnt.p);
  FPC_LAUNCH_CHECK();
  int remaining = read_i32(cnt.p, s);
  // phase 2: join the aggregate of an assigned neighbour (largest root
  // priority), synchronous sweeps
  for (int sweep = 0; remaining > 0; ++sweep) {
    if (sweep > 64) throw Error(FPC_ERR_HIP, "aggregation left nodes");
    k_rk2<<<g, 256, 0, s>>>(agg, roots.p, prio.p, n, key.p);
    k_max_closed<<<g4, 256, 0, s>>>(a.rowptr.p, a.col.p, n, key.p, m1.p);
    FPC_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int), s));
    k_join<<<g, 256, 0, s>>>(iso.p, m1.p, n, agg, cnt.p);
    FPC_LAUNCH_CHECK();
    int r = read_i32(cnt.p, s);
    if (r == remaining) throw Error(FPC_ERR_HIP, "aggregation stalled");
    remaining = r;
  }
  FPC_HIP(hipStreamSynchronize(s));
  return n_agg;
}

void rigid_modes(const double* coords, int64_t n_nodes, int nb, double* B,
                 hipStream_t s) {
  DevBuf<double> part(64 * 6), ctr(3);
  if (coords) {
    k_bbox_partial<<<64, 256, 0, s>>>(coords, n_nodes, part.p);
    k_bbox_final<<<1, 64, 0, s>>>(part.p, 64, ctr.p);
    FPC_LAUNCH_CHECK();
  }
  k_rigid<<<grid_for(n_nodes, 256), 256, 0, s>>>(coords, ctr.p, n_nodes, nb,
                                                 B);
  FPC_LAUNCH_CHECK();
  FPC_HIP(hipStreamSynchronize(s));
}

void tentative(const int32_t* agg, int64_t n_nodes, int64_t n_agg, int bs,
               int nb, const double* B, double drop_tol, double* ptent,
               double* Bc, int32_t* rank, hipStream_t s) {
  if (nb < 1 || nb > 6)
    throw Error(FPC_ERR_ARG, "tentative: 1 to 6 near-nullspace vectors");
  DevBuf<unsigned long long> cnt(n_agg + 1);
  FPC_HIP(hipMemsetAsync(cnt.p, 0, cnt.bytes(), s));
  k_agg_count<<<grid_for(n_nodes, 256), 256, 0, s>>>(agg, n_nodes, cnt.p);
  FPC_LAUNCH_CHECK();
  DevBuf<int64_t> off(n_agg + 1);
  scan_counts((const int64_t*)cnt.p, off.p, n_agg, s);
  DevBuf<unsigned long long> cursor(n_agg + 1);
  FPC_HIP(hipMemcpyAsync(cursor.p, off.p, (n_agg + 1) * sizeof(int64_t),
                         hipMemcpyDeviceToDevice, s));
  DevBuf<int32_t> members(std::max<int64_t>(n_nodes, 1));
  k_agg_fill<<<grid_for(n_nodes, 256), 256, 0, s>>>(agg, n_nodes, cursor.p,
                                                    members.p);
  k_agg_sort<<<grid_for(n_agg, 64), 64, 0, s>>>(off.p, n_agg, bs, TENT_ROWS,
                                                members.p);
  FPC_HIP(hipMemsetAsync(ptent, 0, (size_t)n_nodes * bs * nb * sizeof(double),
                         s));
  if (n_agg) {
    k_tentative_w<1, 4><<<(unsigned)((n_agg + 3) / 4), 256, 0, s>>>(
        off.p, members.p, n_agg, bs, nb, B, drop_tol, ptent, Bc, rank, 0);
    k_tentative_w<4, 8><<<(unsigned)n_agg, 256, 0, s>>>(
        off.p, members.p, n_agg, bs, nb, B, drop_tol, ptent, Bc, rank, 256);
    k_tentative<<<grid_for(n_agg, 64), 64, 0, s>>>(
        off.p, members.p, n_agg, bs, nb, B, drop_tol, ptent, Bc, rank,
        TENT_ROWS);
  }
  FPC_LAUNCH_CHECK();
  FPC_HIP(hipStreamSynchronize(s));
}

void ptent_bsr(const int32_t* agg, int64_t n_nodes, int64_t n_agg, int bs,
               int nb, const double* ptent, Bsr& P, hipStream_t s) {
  P.br = bs;
  P.bc = nb;
  P.nbr = n_nodes;
  P.nbc = n_agg;
  DevBuf<int64_t> cnt(n_nodes);
  k_ptent_count<<<grid_for(n_nodes, 256), 256, 0, s>>>(agg, n_nodes, cnt.p);
  FPC_LAUNCH_CHECK();
  P.rowptr.alloc(n_nodes + 1);
  P.nnzb = scan_counts_total(cnt.p, P.rowptr.p, n_nodes, s);
  P.col.alloc(std::max<int64_t>(P.nnzb, 1));
  P.val.alloc(std::max<int64_t>(P.nnzb * bs * nb, 1));
  k_ptent_fill<<<grid_for(n_nodes, 256), 256, 0, s>>>(
      agg, P.rowptr.p, n_nodes, bs * nb, ptent, P.col.p, P.val.p);
  FPC_LAUNCH_CHECK();
}

void smooth_prolongator(Bsr& AP, const double* dinv, double omega,
                        hipStream_t s) {
  if (AP.nbr == 0) return;
  k_neg_row_scale<<<(unsigned)((AP.nbr + 3) / 4), 256, 0, s>>>(
      AP.rowptr.p, AP.val.p, AP.nbr, AP.br, AP.bc, dinv, omega);
  FPC_LAUNCH_CHECK();
}

void dummy_diag(Bsr& Ac, const int32_t* rank, hipStream_t s) {
  if (Ac.nbr == 0) return;
  k_dummy_diag<<<grid_for(Ac.nbr, 128), 128, 0, s>>>(
      Ac.rowptr.p, Ac.col.p, Ac.val.p, Ac.nbr, Ac.br, rank);
  FPC_LAUNCH_CHECK();
}

void power_start(int64_t n_nodes, int bs, int key_stride,
                 const int32_t* node_rank, double* x, hipStream_t s) {
  k_power_start<<<grid_for(n_nodes * bs, 256), 256, 0, s>>>(
      n_nodes, bs, key_stride, node_rank, x);
  FPC_LAUNCH_CHECK();
}

// D (npad x npad) = [A 0; 0 I] for a row-major n x n A
void dense_pad(const double* A, int64_t n, int64_t npad, double* D,
               hipStream_t s) {
  FPC_HIP(hipMemsetAsync(D, 0, (size_t)npad * npad * sizeof(double), s));
  if (n)
    FPC_HIP(hipMemcpy2DAsync(D, npad * sizeof(double), A, n * sizeof(double),
                             n * sizeof(double), n, hipMemcpyDeviceToDevice,
                             s));
  if (npad > n)
    k_pad_identity<<<grid_for(npad - n, 256), 256, 0, s>>>(D, n, npad);
  FPC_LAUNCH_CHECK();
}

void dense_from_bsr(const Bsr& a, int64_t npad, double* D, hipStream_t s) {
  FPC_HIP(hipMemsetAsync(D, 0, (size_t)npad * npad * sizeof(double), s));
  if (a.nbr)
    k_dense_from_bsr<<<(unsigned)a.nbr, 256, 0, s>>>(
        a.rowptr.p, a.col.p, a.val.p, a.nbr, a.br, a.bc, npad, D);
  const int64_t n = a.nbr * a.br;
  if (npad > n)
    k_pad_identity<<<grid_for(npad - n, 256), 256, 0, s>>>(D, n, npad);
  FPC_LAUNCH_CHECK();
}

// Pivot rows of the panel [o, o + nb) of the n x n matrix D for Gauss-Jordan
// with partial pivoting: LU with partial pivoting of the tall block
// D[o.., o .. o + nb) on a copy (P, (n - o) x nb).  In the elimination the
// rows below the diagonal receive the same updates as in Gauss-Jordan, so
// these are the pivots Gauss-Jordan meets on the swapped matrix.  piv[k] =
// the row of D to exchange with row o + k (LAPACK convention, in order).  A
// column without a nonzero flags FLAG_SINGULAR.  Right-looking and blocked:
// slabs of kLuSlab columns are eliminated column by column (exchanges over
// the whole panel width), then the rows of the slab are solved with its unit
// lower triangle and the rest of the panel takes one rank-kLuSlab update, so
// the panel is read and written once per slab rather than once per column.
constexpr int kLuSlab = 8;
__global__ __launch_bounds__(1024) void k_panel_pivots(
    const double* __restrict__ D, int64_t n, int64_t o, int nb,
    double* __restrict__ P, int32_t* __restrict__ piv, int* flags) {
  __shared__ double s_v[16];
  __shared__ int s_i[16];
  __shared__ double s_l[kLuSlab][kLuSlab];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t m = n - o;
  for (int64_t idx = t; idx < m * nb; idx += 1024) {
    const int64_t r = idx / nb, c = idx - r * nb;
    P[idx] = D[(o + r) * n + o + c];
  }
  __syncthreads();
  for (int s0 = 0; s0 < nb; s0 += kLuSlab) {
    const int s1 = min(s0 + kLuSlab, nb);
    for (int k = s0; k < s1; ++k) {
      double bv = -1.0;
      int bi = k;
      for (int64_t r = k + t; r < m; r += 1024) {
        const double a = fabs(P[r * nb + k]);
        if (a > bv) {
          bv = a;
          bi = (int)r;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        s_v[w] = bv;
        s_i[w] = bi;
      }
      __syncthreads();
      if (t == 0) {
        for (int q = 1; q < 16; ++q)
          if (s_v[q] > s_v[0] || (s_v[q] == s_v[0] && s_i[q] < s_i[0])) {
            s_v[0] = s_v[q];
            s_i[0] = s_i[q];
          }
        piv[k] = (int32_t)(o + s_i[0]);
        if (!(s_v[0] > 0.0) || !isfinite(s_v[0]))
          atomicOr(&flags[FLAG_SINGULAR], 1);
      }
      __syncthreads();
      const int p = s_i[0];
      const bool bad = !(s_v[0] > 0.0) || !isfinite(s_v[0]);
      if (p != k)
        for (int c = t; c < nb; c += 1024) {
          const double x = P[(int64_t)k * nb + c];
          P[(int64_t)k * nb + c] = P[(int64_t)p * nb + c];
          P[(int64_t)p * nb + c] = x;
        }
      __syncthreads();
      // column k of L below the pivot, rank-1 update inside the slab
      const double inv = bad ? 0.0 : 1.0 / P[(int64_t)k * nb + k];
      for (int64_t r = k + 1 + t; r < m; r += 1024) {
        double* __restrict__ row = P + r * nb;
        const double l = row[k] * inv;
        row[k] = l;
        for (int c = k + 1; c < s1; ++c) row[c] -= l * P[(int64_t)k * nb + c];
      }
      __syncthreads();
    }
    if (s1 >= nb) break;
    // rows s0 .. s1 - 1 of U right of the slab: unit lower solve
    if (t < kLuSlab * kLuSlab) {
      const int i = t / kLuSlab, q = t % kLuSlab;
      s_l[i][q] = (s0 + i < s1 && q < i) ? P[(int64_t)(s0 + i) * nb + s0 + q]
                                         : 0.0;
    }
    __syncthreads();
    for (int c = s1 + t; c < nb; c += 1024) {
      double u[kLuSlab];
#pragma unroll
      for (int i = 0; i < kLuSlab; ++i) {
        double v = s0 + i < s1 ? P[(int64_t)(s0 + i) * nb + c] : 0.0;
#pragma unroll
        for (int q = 0; q < i; ++q) v -= s_l[i][q] * u[q];
        u[i] = v;
        if (s0 + i < s1) P[(int64_t)(s0 + i) * nb + c] = v;
      }
    }
    __syncthreads();
    // rank-(s1 - s0) update of the rows below the slab
    const int wr = nb - s1;
    for (int64_t idx = t; idx < (m - s1) * wr; idx += 1024) {
      const int64_t r = s1 + idx / wr;
      const int c = s1 + (int)(idx % wr);
      double* __restrict__ row = P + r * nb;
      double v = row[c];
      for (int q = s0; q < s1; ++q) v -= row[q] * P[(int64_t)q * nb + c];
      row[c] = v;
    }
    __syncthreads();
  }
}

// The same pivots from three kernels per slab of kLuSlabR columns when the
// panel has at most kLuRows rows below the slab's first column: the slab's
// columns are eliminated by one workgroup holding the slab in registers (two
// rows per thread, k_lu_slab), then its exchanges and the unit lower solve
// reach the columns to its right (k_lu_swap_u12, thread per column) and the
// rows below take the rank-kLuSlabR update across the whole grid
// (k_lu_trail).  The column-by-column steps then cost a few barriers each.
constexpr int kLuRows = 2048;
constexpr int kLuSlabR = 16;
__global__ void k_copy_panel(const double* __restrict__ D, int64_t n,
                             int64_t o, int nb, double* __restrict__ P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (n - o) * nb) return;
  const int64_t r = idx / nb, c = idx - r * nb;
  P[idx] = D[(o + r) * n + o + c];
}

// Wavefront maximum of a 64-bit key: DPP exchanges inside each row of 16
// lanes (the two quad swaps, then the half-row and row mirrors leave the
// row's maximum in all its lanes), then the four rows read lane by lane.
// Every lane of the wavefront must be active.
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, 0xf,
                                             0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32),
                                             CTRL, 0xf, 0xf, false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ uint64_t row16_max_u64(uint64_t k) {
  uint64_t o = dpp_u64<0xb1>(k);   // quad_perm [1, 0, 3, 2]
  k = o > k ? o : k;
  o = dpp_u64<0x4e>(k);            // quad_perm [2, 3, 0, 1]
  k = o > k ? o : k;
  o = dpp_u64<0x141>(k);           // row_half_mirror
  k = o > k ? o : k;
  o = dpp_u64<0x140>(k);           // row_mirror
  return o > k ? o : k;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t k) {
  k = row16_max_u64(k);
  uint64_t r = 0;
#pragma unroll
  for (int row = 0; row < 4; ++row) {
    const uint32_t lo =
        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)k, row * 16);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(k >> 32), row * 16);
    const uint64_t v = ((uint64_t)hi << 32) | lo;
    r = v > r ? v : r;
  }
  return r;
}

__device__ __forceinline__ uint64_t lane0_u64(uint64_t k) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(k >> 32), 0)
          << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)k, 0);
}

__global__ __launch_bounds__(1024) void k_lu_slab(double* __restrict__ P,
                                                  int64_t m, int nb, int s0,
                                                  int s1, int64_t o,
                                                  int32_t* __restrict__ piv,
                                                  int* flags) {
  constexpr int W = kLuSlabR;
  static_assert(kLuRows == 2 * 1024, "two rows per thread");
  __shared__ uint64_t s_key[16];
  __shared__ int s_idx[16];
  __shared__ double s_rp[W], s_rq[W];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int rows = (int)(m - s0), ws = s1 - s0;
  const int r0 = t, r1 = t + 1024;
  // rows r0 and r1 of the slab (two arrays, selected by value, so that they
  // stay in registers)
  double A0[W], A1[W];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    A0[c] = (r0 < rows && c < ws) ? P[(int64_t)(s0 + r0) * nb + s0 + c] : 0.0;
    A1[c] = (r1 < rows && c < ws) ? P[(int64_t)(s0 + r1) * nb + s0 + c] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < W; ++q) {
    if (q >= ws) continue;  // uniform: the slab's last columns may be absent
    // largest |entry| of column q at or below row q, first row on ties.
    // Key of a candidate: the bits of |entry| (ordered as integers for
    // nonnegative doubles) plus one, 0 for rows above q or past the end; a
    // thread's row r0 comes before its row r1.
    uint64_t k0 = 0, k1 = 0;
    if (r0 >= q && r0 < rows)
      k0 = (uint64_t)__double_as_longlong(fabs(A0[q])) + 1;
    if (r1 >= q && r1 < rows)
      k1 = (uint64_t)__double_as_longlong(fabs(A1[q])) + 1;
    const bool use1 = k1 > k0;
    const uint64_t key = use1 ? k1 : k0;
    const uint64_t wmax = wave_max_u64(key);
    // the wavefront's first row with the maximum: its rows t precede its
    // rows t + 1024
    const uint64_t m0 = __ballot(key == wmax && !use1);
    const uint64_t m1 = __ballot(key == wmax);
    if (lane == 0) {
      s_key[w] = wmax;
      s_idx[w] = m0 ? 64 * w + __ffsll((unsigned long long)m0) - 1
                    : 1024 + 64 * w + __ffsll((unsigned long long)m1) - 1;
    }
    __syncthreads();
    // the 16 wavefront results, lane i of each row of 16 taking wavefront
    // i's: their maximum, then the first row holding it (rows below 1024
    // first, each half in wavefront order)
    const uint64_t kv = s_key[lane & 15];
    const int iv = s_idx[lane & 15];
    const uint64_t bk = lane0_u64(row16_max_u64(kv));
    const uint64_t t0 = __ballot(kv == bk && iv < 1024) & 0xffffull;
    const uint64_t t1 = __ballot(kv == bk) & 0xffffull;
    const int src = (t0 ? __ffsll((unsigned long long)t0)
                        : __ffsll((unsigned long long)t1)) - 1;
    const int p = __builtin_amdgcn_readlane(iv, src);
    const double pv = __longlong_as_double((long long)(bk - 1));
    const bool bad = bk == 0 || !(pv > 0.0) || !isfinite(pv);
    if (t == 0) {
      piv[s0 + q] = (int32_t)(o + s0 + p);
      if (bad) atomicOr(&flags[FLAG_SINGULAR], 1);
    }
    // the pivot row and row q through LDS, then exchanged (only the
    // wavefronts of the two owners take these branches)
    const bool own_p = t == (p & 1023), p_hi = p >= 1024;
    const bool own_q = t == (q & 1023), q_hi = q >= 1024;
    if (own_p) {
      if (p_hi) {
#pragma unroll
        for (int c = 0; c < W; ++c) s_rp[c] = A1[c];
      } else {
#pragma unroll
        for (int c = 0; c < W; ++c) s_rp[c] = A0[c];
      }
    }
    if (own_q) {
      if (q_hi) {
#pragma unroll
        for (int c = 0; c < W; ++c) s_rq[c] = A1[c];
      } else {
#pragma unroll
        for (int c = 0; c < W; ++c) s_rq[c] = A0[c];
      }
    }
    __syncthreads();
    if (p != q && (own_p || own_q)) {
      // row q takes the pivot row and the pivot row takes row q; a thread
      // may own both (p and q 1024 apart)
      if (own_q && !q_hi) {
#pragma unroll
        for (int c = 0; c < W; ++c) A0[c] = s_rp[c];
      }
      if (own_q && q_hi) {
#pragma unroll
        for (int c = 0; c < W; ++c) A1[c] = s_rp[c];
      }
      if (own_p && !p_hi) {
#pragma unroll
        for (int c = 0; c < W; ++c) A0[c] = s_rq[c];
      }
      if (own_p && p_hi) {
#pragma unroll
        for (int c = 0; c < W; ++c) A1[c] = s_rq[c];
      }
    }
    // column q of L below the pivot, rank-1 update inside the slab
    const double inv = bad ? 0.0 : 1.0 / s_rp[q];
    if (r0 > q && r0 < rows) {
      const double l = A0[q] * inv;
      A0[q] = l;
#pragma unroll
      for (int c = q + 1; c < W; ++c)
        if (c < ws) A0[c] -= l * s_rp[c];
    }
    if (r1 > q && r1 < rows) {
      const double l = A1[q] * inv;
      A1[q] = l;
#pragma unroll
      for (int c = q + 1; c < W; ++c)
        if (c < ws) A1[c] -= l * s_rp[c];
    }
  }
#pragma unroll
  for (int c = 0; c < W; ++c) {
    if (c < ws && r0 < rows) P[(int64_t)(s0 + r0) * nb + s0 + c] = A0[c];
    if (c < ws && r1 < rows) P[(int64_t)(s0 + r1) * nb + s0 + c] = A1[c];
  }
}

// columns c >= s1 of the panel: the slab's exchanges in order, then the
// unit lower solve of its rows
__global__ void k_lu_swap_u12(double* __restrict__ P, int64_t m, int nb,
                              int s0, int s1, int64_t o,
                              const int32_t* __restrict__ piv) {
  const int c = s1 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (c >= nb) return;
  for (int k = s0; k < s1; ++k) {
    const int64_t p = piv[k] - o;
    if (p == k) continue;
    const double x = P[(int64_t)k * nb + c];
    P[(int64_t)k * nb + c] = P[p * nb + c];
    P[p * nb + c] = x;
  }
  double u[kLuSlabR];
#pragma unroll
  for (int i = 0; i < kLuSlabR; ++i) {
    if (s0 + i >= s1) break;
    double v = P[(int64_t)(s0 + i) * nb + c];
    for (int q = 0; q < i; ++q) v -= P[(int64_t)(s0 + i) * nb + s0 + q] * u[q];
    u[i] = v;
    P[(int64_t)(s0 + i) * nb + c] = v;
  }
  (void)m;
}

// rows r >= s1, columns c >= s1: P[r][c] -= sum_q L[r][q] U[q][c]
__global__ void k_lu_trail(double* __restrict__ P, int64_t m, int nb, int s0,
                           int s1) {
  const int c = s1 + (int)(blockIdx.x * 64 + (threadIdx.x & 63));
  const int64_t r = s1 + (int64_t)blockIdx.y * 16 + (threadIdx.x >> 6);
  if (c >= nb || r >= m) return;
  double* __restrict__ row = P + r * nb;
  double v = row[c];
  for (int q = s0; q < s1; ++q) v -= row[q] * P[(int64_t)q * nb + c];
  row[c] = v;
}

// Row exchanges of one panel applied in order to whole rows (thread per
// column).
__global__ void k_swap_rows(double* D, int64_t n, int64_t o, int nb,
                            const int32_t* __restrict__ piv) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int k = 0; k < nb; ++k) {
    const int64_t r = piv[k];
    if (r == o + k) continue;
    const double x = D[(o + k) * n + j];
    D[(o + k) * n + j] = D[r * n + j];
    D[r * n + j] = x;
  }
}

// inv(A) = inv(P A) P: the exchanges applied to the columns in reverse order
// (thread per row).
__global__ void k_unswap_cols(double* D, int64_t n,
                              const int32_t* __restrict__ piv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double* row = D + i * n;
  for (int64_t k = n - 1; k >= 0; --k) {
    const int64_t c = piv[k];
    if (c == k) continue;
    const double x = row[k];
    row[k] = row[c];
    row[c] = x;
  }
}

void gj_inverse(double* D, int64_t n, int* flags, hipStream_t s, bool pivot) {
  if (n % GT) throw Error(FPC_ERR_ARG, "gj_inverse: size not a multiple of 64");
  constexpr int64_t NB = 256;
  DevBuf<int32_t> piv(n);
  DevBuf<double> panel(n * std::min<int64_t>(NB, n));
  // 256-wide panels: copies of the panel row / column feed the panel
  // products, which may not read what they write
  DevBuf<double> prow(NB * n), pcol(n * NB);
  const SkipMap none{INT64_MAX, 0};
  for (int64_t o = 0; o < n; o += NB) {
    const int64_t nb = std::min<int64_t>(NB, n - o);
    // partial pivoting: choose the panel's pivot rows, exchange them
    const int64_t m = n - o;
    if (!pivot) {
      // SPD: diagonal pivots, nonpositive ones flagged by the tile kernel
    } else if (m <= kLuRows) {
      k_copy_panel<<<grid_for(m * nb, 256), 256, 0, s>>>(D, n, o, (int)nb,
                                                         panel.p);
      for (int s0 = 0; s0 < nb; s0 += kLuSlabR) {
        const int s1 = (int)std::min<int64_t>(s0 + kLuSlabR, nb);
        k_lu_slab<<<1, 1024, 0, s>>>(panel.p, m, (int)nb, s0, s1, o,
                                     piv.p + o, flags);
        if (s1 < nb) {
          k_lu_swap_u12<<<grid_for(nb - s1, 64), 64, 0, s>>>(
              panel.p, m, (int)nb, s0, s1, o, piv.p + o);
          const dim3 tg((unsigned)((nb - s1 + 63) / 64),
                        (unsigned)((m - s1 + 15) / 16));
          k_lu_trail<<<tg, 1024, 0, s>>>(panel.p, m, (int)nb, s0, s1);
        }
      }
    } else {
      k_panel_pivots<<<1, 1024, 0, s>>>(D, n, o, (int)nb, panel.p, piv.p + o,
                                        flags);
    }
    if (pivot)
      k_swap_rows<<<grid_for(n, 256), 256, 0, s>>>(D, n, o, (int)nb,
                                                  piv.p + o);
    FPC_LAUNCH_CHECK();
    double* Dkk = D + o * n + o;
    gj_inverse64(Dkk, nb, n, /*spd=*/pivot ? 0 : 1, flags, s);  // Dkk^-1
    if (nb == n) break;
    const SkipMap skip{o, nb};
    FPC_HIP(hipMemcpyAsync(prow.p, D + o * n, nb * n * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    FPC_HIP(hipMemcpy2DAsync(pcol.p, nb * sizeof(double), D + o,
                             n * sizeof(double), nb * sizeof(double), n,
                             hipMemcpyDeviceToDevice, s));
    // row panel: D[o.., j] = Dkk^-1 D[o.., j], j outside the panel
    gemm_f64(nb, n - nb, (int)nb, 1.0, 0.0, Dkk, n, prow.p, n, D + o * n, n,
             none, skip, s);
    // trailing update with the old column panel and the new row panel
    gemm_f64(n - nb, n - nb, (int)nb, -1.0, 1.0, pcol.p, nb, D + o * n, n, D,
             n, skip, skip, s);
    // column panel: D[i, o..] = -D[i, o..] Dkk^-1, i outside the panel
    gemm_f64(n - nb, nb, (int)nb, -1.0, 0.0, pcol.p, nb, Dkk, n, D + o, n,
             skip, none, s);
  }
  if (pivot)
    k_unswap_cols<<<grid_for(n, 256), 256, 0, s>>>(D, n, piv.p);
  FPC_LAUNCH_CHECK();
  FPC_HIP(hipStreamSynchronize(s));
}

void fixed_stress(const Bsr& S1, const Csr& Q1T, const Csr& Q2, double* out,
                  int* flags, hipStream_t s) {
  if (S1.br != 3 || S1.bc != 3) throw Error(FPC_ERR_ARG, "fixed_stress: S1 blocks");
  if (Q2.nrows == 0) return;
  k_fixed_stress<<<(unsigned)Q2.nrows, 64, 0, s>>>(
      S1.rowptr.p, S1.col.p, S1.val.p, Q1T.rowptr.p, Q1T.col.p, Q1T.val.p,
      Q2.rowptr.p, Q2.col.p, Q2.val.p, Q2.nrows, out, flags);
  FPC_LAUNCH_CHECK();
}

void bsr_row_scale_inv_diag(Bsr& b, const Csr& M, double alpha, int* flags,
                            hipStream_t s) {
  if (b.br != 1 || M.nrows != b.nbr) throw Error(FPC_ERR_ARG, "row scaling shape");
  if (!b.nbr) return;
  k_row_scale_inv_diag<<<grid_for(b.nbr, 128), 128, 0, s>>>(
      b.rowptr.p, b.val.p, b.nbr, b.bc, M.rowptr.p, M.col.p, M.val.p, alpha,
      flags);
  FPC_LAUNCH_CHECK();
}

}  // namespace fpc
