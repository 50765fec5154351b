// Sparse setup kernels: validation, scalar CSR products, CSR -> block CSR,
// block add / transpose, row-merge SpGEMM and the sliced-ELL packing used by
// the apply path.
#include "fpc_internal.hpp"

namespace fpc {

namespace {

// ------------------------------------------------------------- validation
// 2^lg lanes per row: lane q checks entries e = a + q, a + q + 2^lg, ...
// (column in range, strictly above the previous entry's, finite value); the
// caller picks lg from the average row length, so that the lanes of a row
// read whole cache lines.
__global__ void k_csr_validate(const int64_t* rowptr, const int32_t* col,
                               const double* val, int64_t nrows,
                               int64_t ncols, int64_t nnz, int lg,
                               int* flags) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t >> lg;
  const int L = 1 << lg;
  const int q = (int)(t & (L - 1));
  if (t == 0 && (rowptr[0] != 0 || rowptr[nrows] != nnz))
    atomicOr(&flags[FLAG_PATTERN], 1);
  if (i >= nrows) return;
  const int64_t a = rowptr[i], b = rowptr[i + 1];
  if (a > b || a < 0 || b > nnz) {
    if (q == 0) atomicOr(&flags[FLAG_PATTERN], 1);
    return;
  }
  bool bad = false, nan = false;
  for (int64_t e = a + q; e < b; e += L) {
    const int32_t c = col[e];
    if (c < 0 || c >= ncols || (e > a && c <= col[e - 1])) bad = true;
    if (!isfinite(val[e])) nan = true;
  }
  if (bad) atomicOr(&flags[FLAG_PATTERN], 1);
  if (nan) atomicOr(&flags[FLAG_NAN], 1);
}

// ------------------------------------------------------------- CSR SpMV
__global__ void k_csr_spmv2(const int64_t* rp1, const int32_t* c1,
                            const double* v1, const double* x1, double a1,
                            const int64_t* rp2, const int32_t* c2,
                            const double* v2, const double* x2, double a2,
                            double* y, double beta, int64_t nrows) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  const double s1 = csr_row_sum(c1, v1, x1, rp1[i], rp1[i + 1]);
  double r = a1 * s1;
  if (rp2) {
    const double s2 = csr_row_sum(c2, v2, x2, rp2[i], rp2[i + 1]);
    r += a2 * s2;
  }
  y[i] = (beta == 0.0) ? r : beta * y[i] + r;
}

// Products of one or two CSR matrices over a row list (rows where m1 is
// nonempty, or with skip1 the rows of m2's list where m1 is empty), the same
// arithmetic per row as k_csr_spmv2: y = beta y + a1 (m1 x1) + a2 (m2 x2).
__global__ void k_csr_spmv2_rows(const int32_t* rows, int64_t nr, int skip1,
                                 const int64_t* rp1, const int32_t* c1,
                                 const double* v1, const double* x1, double a1,
                                 const int64_t* rp2, const int32_t* c2,
                                 const double* v2, const double* x2, double a2,
                                 double* y, double beta) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nr) return;
  const int64_t i = rows[t];
  if (skip1 && rp1 && rp1[i] < rp1[i + 1]) return;
  double s1 = 0.0;
  if (rp1)
    s1 = csr_row_sum(c1, v1, x1, rp1[i], rp1[i + 1]);
  double r = a1 * s1;
  if (rp2) {
    const double s2 = csr_row_sum(c2, v2, x2, rp2[i], rp2[i + 1]);
    r += a2 * s2;
  }
  y[i] = (beta == 0.0) ? r : beta * y[i] + r;
}

// Several row sets of csr_spmv2 in one launch: job q covers threads
// [start[q], start[q + 1]) and does, per row, the arithmetic of
// k_csr_spmv2 (rows == nullptr: thread t is row t) or of k_csr_spmv2_rows.
struct Spmv2Job {
  const int32_t* rows;
  int skip1;
  const int64_t* rp1;
  const int32_t* c1;
  const double* v1;
  const double* x1;
  double a1;
  const int64_t* rp2;
  const int32_t* c2;
  const double* v2;
  const double* x2;
  double a2;
  double* y;
  double beta;
};
constexpr int kSpmv2Jobs = 8;
struct Spmv2Jobs {
  Spmv2Job j[kSpmv2Jobs];
  int64_t start[kSpmv2Jobs + 1];
  int n;
};

__global__ void k_csr_spmv2_multi(const Spmv2Jobs jobs) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= jobs.start[jobs.n]) return;
  int q = 0;
  while (t >= jobs.start[q + 1]) ++q;
  const Spmv2Job& J = jobs.j[q];
  const int64_t r = t - jobs.start[q];
  const int64_t i = J.rows ? J.rows[r] : r;
  if (J.skip1 && J.rp1 && J.rp1[i] < J.rp1[i + 1]) return;
  double s1 = 0.0;
  if (J.rp1)
    s1 = csr_row_sum(J.c1, J.v1, J.x1, J.rp1[i], J.rp1[i + 1]);
  double res = J.a1 * s1;
  if (J.rp2) {
    const double s2 = csr_row_sum(J.c2, J.v2, J.x2, J.rp2[i], J.rp2[i + 1]);
    res += J.a2 * s2;
  }
  J.y[i] = (J.beta == 0.0) ? res : J.beta * J.y[i] + res;
}

__global__ void k_row_nonempty(const int64_t* rp, int64_t n, int64_t* f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = rp[i] < rp[i + 1] ? 1 : 0;
}

__global__ void k_row_list(const int64_t* f, const int64_t* scan, int64_t n,
                           int32_t* list) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && f[i]) list[scan[i]] = (int32_t)i;
}

// ------------------------------------------------------------- transpose
__global__ void k_col_count(const int64_t* rowptr, const int32_t* col,
                            int64_t nrows, unsigned long long* cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
    atomicAdd(&cnt[col[e]], 1ull);
}

__global__ void k_tr_fill(const int64_t* rowptr, const int32_t* col,
                          int64_t nrows, unsigned long long* cursor,
                          int32_t* colT, int64_t* src) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    unsigned long long pos = atomicAdd(&cursor[col[e]], 1ull);
    colT[pos] = (int32_t)i;
    src[pos] = e;
  }
}

// Rows of the transpose up to RS entries: one wavefront per row ranks its
// entries in LDS (keys are distinct) and writes them in order.
constexpr int RS = 4096;
__global__ __launch_bounds__(64) void k_tr_sort_wave(const int64_t* rowptrT,
                                                     int64_t nrowsT,
                                                     int32_t* colT,
                                                     int64_t* src) {
  __shared__ int32_t kc[RS];
  __shared__ int64_t ks[RS];
  const int64_t r = blockIdx.x;
  const int lane = threadIdx.x;
  if (r >= nrowsT) return;
  const int64_t a = rowptrT[r];
  const int n = (int)(rowptrT[r + 1] - a);
  if (n < 2 || n > RS) return;
  for (int e = lane; e < n; e += 64) {
    kc[e] = colT[a + e];
    ks[e] = src[a + e];
  }
  __syncthreads();
  for (int e = lane; e < n; e += 64) {
    const int32_t key = kc[e];
    int rank = 0;
    for (int f = 0; f < n; ++f) rank += (kc[f] < key);
    colT[a + rank] = key;
    src[a + rank] = ks[e];
  }
}

__global__ void k_tr_sort_long(const int64_t* rowptrT, int64_t nrowsT,
                               int32_t* colT, int64_t* src) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrowsT) return;
  int64_t a = rowptrT[r], b = rowptrT[r + 1];
  if (b - a <= RS) return;
  for (int64_t e = a + 1; e < b; ++e) {
    int32_t c = colT[e];
    int64_t s = src[e];
    int64_t f = e - 1;
    while (f >= a && colT[f] > c) {
      colT[f + 1] = colT[f];
      src[f + 1] = src[f];
      --f;
    }
    colT[f + 1] = c;
    src[f + 1] = s;
  }
}

// One thread per value of the transposed blocks (consecutive threads write
// consecutive values; a block's values are read from one source block).
template <int BR, int BC>
__global__ void k_tr_gather(const double* val, const int64_t* src,
                            int64_t nnzb, double* valT) {
  constexpr int B = BR * BC;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnzb * B) return;
  const int64_t p = e / B;
  const int q = (int)(e - p * B);
  const int c = q / BR, r = q - c * BR;   // valT block is BC x BR
  valT[e] = val[src[p] * B + r * BC + c];
}

// ------------------------------------------------------------- CSR -> BSR
// Entries of a block row (its BR scalar rows) held in LDS by k_to_bsr_w.
constexpr int TB_CAP = 512;

__device__ inline int64_t block_row_entries(const int64_t* rowptr,
                                            int64_t nrows, int64_t I, int br) {
  const int64_t r0 = I * br, r1 = min(nrows, r0 + br);
  return rowptr[r1] - rowptr[r0];
}

// First index in [lo, hi) of the sorted LDS list v whose value is >= b.
__device__ inline int lds_lower_bound(const int32_t* v, int lo, int hi,
                                      int32_t b) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (v[mid] < b) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// One wavefront per block row with at most TB_CAP scalar entries (the BR
// rows concatenated, each sorted by column).  Entry k with block column b
// is the first of b if it starts b in its own row and no earlier row holds
// b (binary searches in LDS); gp is the exclusive prefix count of first
// entries.  The block of b sits at the number of distinct block columns
// below b, which is the sum over rows q of the first entries of q below b:
// gp at the lower bound of b in row q minus gp at the start of q.  Count
// mode (bcol null) writes the number of blocks, fill mode the blocks.
template <int BR, int BC>
__global__ __launch_bounds__(64) void k_to_bsr_w(
    const int64_t* rowptr, const int32_t* col, const double* val,
    int64_t nrows, const int64_t* browptr, int64_t* bcount, int32_t* bcol,
    double* bval) {
  __shared__ int32_t sbc[TB_CAP];
  __shared__ int32_t gp[TB_CAP + 1];
  const int64_t I = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t r0 = I * BR;
  const int nr = (int)min<int64_t>(BR, nrows - r0);
  const int64_t a = rowptr[r0];
  const int m = (int)(rowptr[r0 + nr] - a);
  if (m > TB_CAP) return;  // done by k_to_bsr
  int rs[BR + 1];
#pragma unroll
  for (int q = 0; q <= BR; ++q)
    rs[q] = (int)(rowptr[r0 + (q < nr ? q : nr)] - a);
  // the BR rows are contiguous in the CSR arrays: entry k is col[a + k]
  for (int k = lane; k < m; k += 64) sbc[k] = col[a + k] / BC;
  __syncthreads();
  // first flags, then their exclusive prefix over 64-entry chunks
  int carry = 0;
  for (int k0 = 0; k0 < m; k0 += 64) {
    const int k = k0 + lane;
    bool first = false;
    if (k < m) {
      int r = 0;
#pragma unroll
      for (int q = 1; q < BR; ++q)
        if (q < nr && k >= rs[q]) r = q;
      const int32_t b = sbc[k];
      first = k == rs[r] || sbc[k - 1] != b;
#pragma unroll
      for (int q = 0; q < BR - 1; ++q)
        if (q < r && first) {
          const int p = lds_lower_bound(sbc, rs[q], rs[q + 1], b);
          first = !(p < rs[q + 1] && sbc[p] == b);
        }
    }
    const uint64_t mask = __ballot(first);
    if (k < m)
      gp[k] = carry + __popcll(mask & ((uint64_t(1) << lane) - 1));
    carry += __popcll(mask);
  }
  if (lane == 0) gp[m] = carry;
  __syncthreads();
  if (!bcol) {
    if (lane == 0) bcount[I] = carry;
    return;
  }
  const int64_t out = browptr[I];
  for (int k = lane; k < m; k += 64) {
    const int32_t b = sbc[k];
    int r = 0;
#pragma unroll
    for (int q = 1; q < BR; ++q)
      if (q < nr && k >= rs[q]) r = q;
    int rank = 0;
#pragma unroll
    for (int q = 0; q < BR; ++q)
      if (q < nr) {
        const int p = lds_lower_bound(sbc, rs[q], rs[q + 1], b);
        rank += gp[p] - gp[rs[q]];
      }
    const bool first = gp[k + 1] != gp[k];
    if (first) bcol[out + rank] = b;
    bval[(out + rank) * (BR * BC) + r * BC + col[a + k] % BC] = val[a + k];
  }
}

// Thread per block row (merge of its BR scalar rows); with min_m, only the
// block rows with more than min_m scalar entries.
template <int BR, int BC>
__global__ void k_to_bsr(const int64_t* rowptr, const int32_t* col,
                         const double* val, int64_t nrows, int64_t nbr,
                         const int64_t* browptr, int64_t* bcount,
                         int32_t* bcol, double* bval, int64_t min_m) {
  int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nbr) return;
  if (block_row_entries(rowptr, nrows, I, BR) <= min_m) return;
  int64_t p[BR], e[BR];
#pragma unroll
  for (int r = 0; r < BR; ++r) {
    int64_t row = I * BR + r;
    p[r] = row < nrows ? rowptr[row] : 0;
    e[r] = row < nrows ? rowptr[row + 1] : 0;
  }
  int64_t n = 0;
  int64_t out = browptr ? browptr[I] : 0;
  while (true) {
    int32_t m = 0x7fffffff;
#pragma unroll
    for (int r = 0; r < BR; ++r)
      if (p[r] < e[r]) m = min(m, col[p[r]] / BC);
    if (m == 0x7fffffff) break;
    if (bcol) {
      bcol[out + n] = m;
      double* blk = bval + (out + n) * (BR * BC);
#pragma unroll
      for (int r = 0; r < BR; ++r)
        while (p[r] < e[r] && col[p[r]] / BC == m) {
          blk[r * BC + (col[p[r]] % BC)] = val[p[r]];
          ++p[r];
        }
    } else {
#pragma unroll
      for (int r = 0; r < BR; ++r)
        while (p[r] < e[r] && col[p[r]] / BC == m) ++p[r];
    }
    ++n;
  }
  if (bcount) bcount[I] = n;
}

// ------------------------------------------------------------- BSR add
// Count pass of C = A + B: blocks in the union of the two sorted rows.
__global__ void k_bsr_add_count(const int64_t* ra, const int32_t* ca,
                                const int64_t* rb, const int32_t* cb,
                                int64_t nbr, int64_t* cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbr) return;
  int64_t pa = ra[i], ea = ra[i + 1], pb = rb[i], eb = rb[i + 1];
  int64_t n = 0;
  while (pa < ea || pb < eb) {
    int32_t x = pa < ea ? ca[pa] : 0x7fffffff;
    int32_t y = pb < eb ? cb[pb] : 0x7fffffff;
    int32_t m = min(x, y);
    if (x == m) ++pa;
    if (y == m) ++pb;
    ++n;
  }
  cnt[i] = n;
}

// Fill pass of C = A + B with one wavefront per block row: a row with one
// source is a contiguous copy; otherwise the two column lists are staged in
// LDS, lane 0 merges them into (source index, source index) pairs and the
// wavefront writes the merged blocks.  Rows longer than the LDS lists merge
// serially on lane 0.  The sums are formed as in k_bsr_add.
constexpr int ADD_CAP = 256;

template <int B>
__device__ inline void bsr_add_row_serial(const int32_t* ca, const double* va,
                                          const int32_t* cb, const double* vb,
                                          int64_t pa, int64_t ea, int64_t pb,
                                          int64_t eb, int64_t out, int32_t* cc,
                                          double* vc) {
  int64_t n = 0;
  while (pa < ea || pb < eb) {
    const int32_t x = pa < ea ? ca[pa] : 0x7fffffff;
    const int32_t y = pb < eb ? cb[pb] : 0x7fffffff;
    const int32_t m = min(x, y);
    cc[out + n] = m;
    double* o = vc + (out + n) * B;
    for (int q = 0; q < B; ++q) {
      double v = 0.0;
      if (x == m) v += va[pa * B + q];
      if (y == m) v += vb[pb * B + q];
      o[q] = v;
    }
    if (x == m) ++pa;
    if (y == m) ++pb;
    ++n;
  }
}

template <int B>
__global__ __launch_bounds__(256) void k_bsr_add_w(
    const int64_t* __restrict__ ra, const int32_t* __restrict__ ca,
    const double* __restrict__ va, const int64_t* __restrict__ rb,
    const int32_t* __restrict__ cb, const double* __restrict__ vb, int64_t nbr,
    const int64_t* __restrict__ rc, int32_t* __restrict__ cc,
    double* __restrict__ vc) {
  __shared__ int32_t sa[4][ADD_CAP], sb[4][ADD_CAP];
  __shared__ int32_t oa[4][2 * ADD_CAP], ob[4][2 * ADD_CAP];
  __shared__ int32_t scount[4];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + w;
  const bool valid = i < nbr;
  int64_t pa = 0, ea = 0, pb = 0, eb = 0, out = 0;
  if (valid) {
    pa = ra[i];
    ea = ra[i + 1];
    pb = rb[i];
    eb = rb[i + 1];
    out = rc[i];
  }
  const int64_t na = ea - pa, nb = eb - pb;
  const bool single = valid && (na == 0 || nb == 0);
  const bool big = valid && !single && (na > ADD_CAP || nb > ADD_CAP);
  const bool staged = valid && !single && !big;
  if (single) {
    const bool fromA = nb == 0;
    const int64_t p = fromA ? pa : pb, len = fromA ? na : nb;
    const int32_t* __restrict__ cs = fromA ? ca : cb;
    const double* __restrict__ vs = fromA ? va : vb;
    // a one-source sum is 0.0 + value, as in the merge
    for (int64_t e = lane; e < len; e += 64) cc[out + e] = cs[p + e];
    for (int64_t e = lane; e < len * B; e += 64) vc[out * B + e] = 0.0 + vs[p * B + e];
  }
  if (big && lane == 0) bsr_add_row_serial<B>(ca, va, cb, vb, pa, ea, pb, eb, out, cc, vc);
  if (staged) {
    for (int64_t e = lane; e < na; e += 64) sa[w][e] = ca[pa + e];
    for (int64_t e = lane; e < nb; e += 64) sb[w][e] = cb[pb + e];
  }
  __syncthreads();
  if (staged && lane == 0) {
    int ka = 0, kb = 0, n = 0;
    while (ka < na || kb < nb) {
      const int32_t x = ka < na ? sa[w][ka] : 0x7fffffff;
      const int32_t y = kb < nb ? sb[w][kb] : 0x7fffffff;
      const int32_t m = min(x, y);
      oa[w][n] = x == m ? ka : -1;
      ob[w][n] = y == m ? kb : -1;
      if (x == m) ++ka;
      if (y == m) ++kb;
      ++n;
    }
    scount[w] = n;
  }
  __syncthreads();
  if (staged) {
    const int n = scount[w];
    for (int e = lane; e < n; e += 64) {
      const int ja = oa[w][e], jb = ob[w][e];
      cc[out + e] = ja >= 0 ? sa[w][ja] : sb[w][jb];
    }
    for (int e = lane; e < n * B; e += 64) {
      const int o = e / B, q = e - o * B;
      const int ja = oa[w][o], jb = ob[w][o];
      double v = 0.0;
      if (ja >= 0) v += va[(pa + ja) * B + q];
      if (jb >= 0) v += vb[(pb + jb) * B + q];
      vc[(out + o) * B + q] = v;
    }
  }
}

// ------------------------------------------------------------- SpGEMM
// The hash table of a row lives in LDS; its size (a power of two, at most
// 4096 slots) is twice the largest possible row length of A*B (the sum of
// the B row lengths over an A row), so small products run at high occupancy.
constexpr int HS_MAX_BITS = 12;

__device__ inline int hslot(int c, int bits) {
  return (int)(((uint32_t)c * 2654435761u) >> (32 - bits));
}

__device__ inline bool hinsert(int* tab, int bits, int* ucount, int c) {
  const int hs = 1 << bits;
  int h = hslot(c, bits);
  for (int probe = 0; probe < hs; ++probe) {
    int old = atomicCAS(&tab[h], -1, c);
    if (old == -1) {
      atomicAdd(ucount, 1);
      return true;
    }
    if (old == c) return true;
    h = (h + 1) & (hs - 1);
  }
  return false;
}

// out = max over rows of sum_{k in row of A} |row k of B| (upper bound on
// the row length of A*B)
__global__ void k_spgemm_bound(const int64_t* ra, const int32_t* ca,
                               const int64_t* rb, int64_t nrows,
                               unsigned long long* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  unsigned long long t = 0;
  for (int64_t e = ra[i]; e < ra[i + 1]; ++e)
    t += (unsigned long long)(rb[ca[e] + 1] - rb[ca[e]]);
  atomicMax(out, t);
}

__global__ void k_max_count(const int64_t* cnt, int64_t n,
                            unsigned long long* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicMax(out, (unsigned long long)cnt[i]);
}

// One 64-thread block per row: hash the block columns of the row of A*B;
// phase 0 counts them, phase 1 writes them sorted.
__global__ __launch_bounds__(64) void k_spgemm_sym(
    const int64_t* ra, const int32_t* ca, const int64_t* rb,
    const int32_t* cb, int64_t nrows, const int64_t* rc, int64_t* cnt,
    int32_t* cc, int* flags, int bits) {
  extern __shared__ int dyn[];
  __shared__ int ucount;
  __shared__ int fail;
  __shared__ int64_t pstart[64];
  __shared__ int pend[64];
  const int hs = 1 << bits;
  int* tab = dyn;
  int* lst = dyn + hs;
  const int64_t row = blockIdx.x;
  const int lane = threadIdx.x;
  if (row >= nrows) return;
  for (int s = lane; s < hs; s += 64) tab[s] = -1;
  if (lane == 0) {
    ucount = 0;
    fail = 0;
  }
  __syncthreads();
  // up to 64 A entries at a time; their (A entry, B entry) pairs are spread
  // over the lanes through an inclusive scan of the B row lengths
  const int64_t aend = ra[row + 1];
  for (int64_t ea0 = ra[row]; ea0 < aend; ea0 += 64) {
    const int64_t ea = ea0 + lane;
    int len = 0;
    int64_t st = 0;
    if (ea < aend) {
      const int32_t k = ca[ea];
      st = rb[k];
      len = (int)(rb[k + 1] - st);
    }
    int incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    pstart[lane] = st;
    pend[lane] = incl;
    const int total = __shfl(incl, 63, 64);
    __syncthreads();
    for (int p = lane; p < total; p += 64) {
      int lo = 0, hi = 63;  // first entry with pend > p
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (pend[mid] > p) hi = mid;
        else lo = mid + 1;
      }
      const int off = p - (lo ? pend[lo - 1] : 0);
      if (!hinsert(tab, bits, &ucount, cb[pstart[lo] + off])) fail = 1;
    }
    __syncthreads();
    if (ucount > (hs * 3) / 4) fail = 1;
    if (fail) break;
  }
  __syncthreads();
  if (fail) {
    if (lane == 0) {
      atomicOr(&flags[FLAG_OVERFLOW], 1);
      if (cnt) cnt[row] = 0;
    }
    return;
  }
  if (cnt) {
    if (lane == 0) cnt[row] = ucount;
    return;
  }
  // compact the occupied slots, then rank-sort into the output row
  int base = 0;
  for (int s0 = 0; s0 < hs; s0 += 64) {
    int c = s0 + lane < hs ? tab[s0 + lane] : -1;
    bool v = c >= 0;
    unsigned long long m = __ballot(v);
    int before = __popcll(m & ((1ull << lane) - 1ull));
    if (v) lst[base + before] = c;
    base += __popcll(m);
  }
  __syncthreads();
  const int n = base;
  const int64_t out = rc[row];
  for (int e = lane; e < n; e += 64) {
    int c = lst[e];
    int r = 0;
    for (int f = 0; f < n; ++f) r += (lst[f] < c);
    cc[out + r] = c;
  }
}

// One step of a row of the numeric phase below: the entries eb of B's row
// k (lane group le takes eb = b0 + le, b0 + le + EPP, ...) times the A
// block a, added to the row's accumulator blocks in LDS (distinct entries
// of one B row hit distinct output blocks).
template <int BM, int BK, int BN>
__device__ inline void spgemm_step(const double (&a)[BM * BK], int64_t b0,
                                   int64_t bend, const int32_t* cb,
                                   const double* vb, const int* scol, int clen,
                                   double* sacc, int le, int c) {
  constexpr int EPP = 64 / BN;
  for (int64_t eb = b0 + le; le < EPP && eb < bend; eb += EPP) {
    const int32_t j = cb[eb];
    // the B values are loaded before the search for the output slot, so
    // their latency overlaps it (the entry exists: eb < bend)
    const double* b = vb + eb * (BK * BN) + c;
    double bt[BK];
#pragma unroll
    for (int t = 0; t < BK; ++t) bt[t] = b[t * BN];
    int lo = 0, hi = clen;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (scol[mid] < j) lo = mid + 1;
      else hi = mid;
    }
    if (lo >= clen || scol[lo] != j) continue;
    double* o = sacc + lo * (BM * BN) + c;
#pragma unroll
    for (int r = 0; r < BM; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < BK; ++t) acc += a[r * BK + t] * bt[t];
      o[r * BN] += acc;
    }
  }
}

// Numeric phase with the output row accumulated in LDS (cap blocks at
// most).  Lane (e, c) = (lane / BN, lane % BN) takes block column c of B
// entry e of each group of 64 / BN entries; the entries of A's row are taken
// one after the other (a barrier between them), so per output value the
// terms are added in the order of k_spgemm_num below (A entries ascending),
// with one global write per output value.  For 3x3 A blocks (A P_tent
// and A P on the finest level, short B rows) the entries are taken SA at a
// time with their B-row bounds and values staged in LDS by parallel loads,
// so the walk over them waits only for B's entries; for the long rows of
// R (A P) that staging cost more than it saved.
template <int BM, int BK, int BN>
__global__ __launch_bounds__(64) void k_spgemm_num_lds(
    const int64_t* ra, const int32_t* ca, const double* va, const int64_t* rb,
    const int32_t* cb, const double* vb, int64_t nrows, const int64_t* rc,
    const int32_t* cc, double* vc, int cap) {
  constexpr bool kStage = BM * BK <= 9;
  constexpr int SA = kStage ? 16 : 1;
  __shared__ double s_a[SA][BM * BK];
  __shared__ int64_t s_b0[SA], s_b1[SA];
  extern __shared__ double sacc[];
  int* scol = (int*)(sacc + (int64_t)cap * BM * BN);
  const int64_t row = blockIdx.x;
  const int lane = threadIdx.x;
  const int le = lane / BN, c = lane % BN;
  if (row >= nrows) return;
  const int64_t c0 = rc[row];
  const int clen = (int)(rc[row + 1] - c0);
  for (int q = lane; q < clen * BM * BN; q += 64) sacc[q] = 0.0;
  for (int q = lane; q < clen; q += 64) scol[q] = cc[c0 + q];
  const int64_t a0 = ra[row], a1 = ra[row + 1];
  if constexpr (!kStage) {
    __syncthreads();
    for (int64_t ea = a0; ea < a1; ++ea) {
      const int32_t k = ca[ea];
      double a[BM * BK];
#pragma unroll
      for (int q = 0; q < BM * BK; ++q) a[q] = va[ea * (BM * BK) + q];
      spgemm_step<BM, BK, BN>(a, rb[k], rb[k + 1], cb, vb, scol, clen, sacc,
                              le, c);
      __syncthreads();
    }
  } else {
    for (int64_t e0 = a0; e0 < a1; e0 += SA) {
      const int na = (int)(a1 - e0 < SA ? a1 - e0 : SA);
      __syncthreads();  // the previous chunk is done with the staging arrays
      if (lane < na) {
        const int32_t k = ca[e0 + lane];
        s_b0[lane] = rb[k];
        s_b1[lane] = rb[k + 1];
      }
      for (int q = lane; q < na * BM * BK; q += 64)
        s_a[q / (BM * BK)][q % (BM * BK)] = va[e0 * (BM * BK) + q];
      __syncthreads();
      for (int e = 0; e < na; ++e) {
        double a[BM * BK];
#pragma unroll
        for (int q = 0; q < BM * BK; ++q) a[q] = s_a[e][q];
        spgemm_step<BM, BK, BN>(a, s_b0[e], s_b1[e], cb, vb, scol, clen, sacc,
                                le, c);
        __syncthreads();
      }
    }
  }
  __syncthreads();
  for (int q = lane; q < clen * BM * BN; q += 64) vc[c0 * BM * BN + q] = sacc[q];
}

// Numeric phase when every row of B holds at most one block (A P_tent):
// each entry of A's row meets one output block, so the products of up to
// NE entries are formed at once (lane = (entry, block column)) and staged
// in LDS with their output slots; lane q then adds, for its output values,
// the staged products in entry order.  Every output value is the sum of its
// terms in ascending A order, each term summed over t first, as in the
// kernels above: the results are the same bit for bit.  Output rows of up
// to 64 QM / (BM BN) blocks (the caller checks).
template <int BM, int BK, int BN, int QM>
__global__ __launch_bounds__(64) void k_spgemm_num_b1(
    const int64_t* ra, const int32_t* ca, const double* va, const int64_t* rb,
    const int32_t* cb, const double* vb, int64_t nrows, const int64_t* rc,
    const int32_t* cc, double* vc, int* flags) {
  constexpr int NE = 32;
  __shared__ double s_p[NE][BM * BN];
  __shared__ int s_t[NE];
  __shared__ int scol[64 * QM / (BM * BN)];
  const int64_t row = blockIdx.x;
  const int lane = threadIdx.x;
  if (row >= nrows) return;
  const int64_t c0 = rc[row];
  const int clen = (int)(rc[row + 1] - c0);
  const int nout = clen * BM * BN;
  for (int q = lane; q < clen; q += 64) scol[q] = cc[c0 + q];
  double acc[QM];
#pragma unroll
  for (int i = 0; i < QM; ++i) acc[i] = 0.0;
  const int64_t a0 = ra[row], a1 = ra[row + 1];
  for (int64_t e0 = a0; e0 < a1; e0 += NE) {
    const int ne = (int)(a1 - e0 < NE ? a1 - e0 : NE);
    __syncthreads();  // scol written; the previous chunk's products used
    for (int w = lane; w < ne * BN; w += 64) {
      const int e = w / BN, cj = w % BN;
      const int64_t ea = e0 + e;
      const int32_t k = ca[ea];
      const int64_t b0 = rb[k];
      const int64_t b1 = rb[k + 1];
      const bool has = b0 < b1;
      if (b1 - b0 > 1) atomicOr(&flags[FLAG_PATTERN], 1);  // not one block
      if (cj == 0) {
        int slot = -1;
        if (has) {
          const int32_t j = cb[b0];
          int lo = 0, hi = clen;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (scol[mid] < j) lo = mid + 1;
            else hi = mid;
          }
          if (lo < clen && scol[lo] == j) slot = lo;
        }
        s_t[e] = slot;
      }
#pragma unroll
      for (int r = 0; r < BM; ++r) {
        double t = 0.0;
        if (has)
#pragma unroll
          for (int u = 0; u < BK; ++u)
            t += va[ea * (BM * BK) + r * BK + u] * vb[b0 * (BK * BN) + u * BN + cj];
        s_p[e][r * BN + cj] = t;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < QM; ++i) {
      const int q = lane + 64 * i;
      if (q < nout) {
        const int slot = q / (BM * BN), rq = q % (BM * BN);
        for (int e = 0; e < ne; ++e)
          if (s_t[e] == slot) acc[i] += s_p[e][rq];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < QM; ++i) {
    const int q = lane + 64 * i;
    if (q < nout) vc[c0 * BM * BN + q] = acc[i];
  }
}

// Numeric phase: C row i = sum_k A(i,k) B(k,:).  The loop over the entries
// of A's row is sequential; within one step the lanes take distinct entries
// of B's row, hence distinct output blocks, so the accumulation order is
// fixed and race free.
template <int BM, int BK, int BN>
__global__ __launch_bounds__(64) void k_spgemm_num(
    const int64_t* ra, const int32_t* ca, const double* va, const int64_t* rb,
    const int32_t* cb, const double* vb, int64_t nrows, const int64_t* rc,
    const int32_t* cc, double* vc) {
  const int64_t row = blockIdx.x;
  const int lane = threadIdx.x;
  if (row >= nrows) return;
  const int64_t c0 = rc[row];
  const int clen = (int)(rc[row + 1] - c0);
  for (int64_t q = lane; q < (int64_t)clen * BM * BN; q += 64)
    vc[c0 * BM * BN + q] = 0.0;
  __syncthreads();
  const int32_t* crow = cc + c0;
  for (int64_t ea = ra[row]; ea < ra[row + 1]; ++ea) {
    const int32_t k = ca[ea];
    double a[BM * BK];
#pragma unroll
    for (int q = 0; q < BM * BK; ++q) a[q] = va[ea * (BM * BK) + q];
    for (int64_t eb = rb[k] + lane; eb < rb[k + 1]; eb += 64) {
      const int32_t j = cb[eb];
      int lo = 0, hi = clen;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (crow[mid] < j) lo = mid + 1;
        else hi = mid;
      }
      if (lo >= clen || crow[lo] != j) continue;  // cannot happen: pattern
                                                  // comes from the same hash
      const double* b = vb + eb * (BK * BN);
      double* o = vc + (c0 + lo) * (BM * BN);
#pragma unroll
      for (int r = 0; r < BM; ++r)
#pragma unroll
        for (int c = 0; c < BN; ++c) {
          double acc = 0.0;
#pragma unroll
          for (int t = 0; t < BK; ++t) acc += a[r * BK + t] * b[t * BN + c];
          o[r * BN + c] += acc;
        }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------- BSR -> SELL
// Slots of each slice: its longest row times the slice height (perm: the
// row at each position, null for the identity).
__global__ void k_slice_len(const int64_t* rowptr, const int32_t* perm,
                            int64_t nrows, int64_t nslices, int64_t* slots) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslices) return;
  int64_t m = 0;
  for (int l = 0; l < kSliceH; ++l) {
    int64_t p = s * kSliceH + l;
    if (p >= nrows) break;
    const int64_t r = perm ? (int64_t)perm[p] : p;
    m = max(m, rowptr[r + 1] - rowptr[r]);
  }
  slots[s] = m * kSliceH;
}

// Rows sorted by length (longest first, ties by index) within windows of
// kSortW rows, so that a slice holds rows of similar length and pads less:
// perm[position] = row, pos[row] = position.
constexpr int kSortW = 2048, kSortT = 512;
__global__ __launch_bounds__(kSortT) void k_window_sort(
    const int64_t* __restrict__ rowptr, int64_t nrows, int32_t* __restrict__ perm,
    int32_t* __restrict__ pos) {
  __shared__ int64_t slen[kSortW];
  const int64_t w0 = (int64_t)blockIdx.x * kSortW;
  const int nw = (int)min<int64_t>(kSortW, nrows - w0);
  for (int i = threadIdx.x; i < kSortW; i += kSortT)
    slen[i] = i < nw ? rowptr[w0 + i + 1] - rowptr[w0 + i] : -1;
  __syncthreads();
  for (int i = threadIdx.x; i < nw; i += kSortT) {
    const int64_t len = slen[i];
    int rank = 0;
    for (int j = 0; j < nw; ++j) {
      const int64_t lj = slen[j];
      rank += (lj > len) || (lj == len && j < i);
    }
    perm[w0 + rank] = (int32_t)(w0 + i);
    pos[w0 + i] = (int32_t)(w0 + rank);
  }
}

// 3x3 blocks whose row and column i0 are zero off the diagonal (a zero
// pattern that is common in stiffness blocks) are stored as five values,
// (m[i0][i0], m[i1][i1], m[i1][i2], m[i2][i1], m[i2][i2]) with i1 < i2 the
// other two indices, in the first five value planes of their slot; the class
// (0 full, 1 + i0 packed) sits in bits 30-31 of the column index.
__device__ inline int class33(const double* v) {
#pragma unroll
  for (int i0 = 0; i0 < 3; ++i0) {
    bool zero = true;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (j != i0) zero = zero && v[i0 * 3 + j] == 0.0 && v[j * 3 + i0] == 0.0;
    if (zero) return 1 + i0;
  }
  return 0;
}

__device__ inline void pack33(const double* v, int cls, double* p) {
  const int i0 = cls - 1;
  const int i1 = i0 == 0 ? 1 : 0, i2 = i0 == 2 ? 1 : 2;
  p[0] = v[i0 * 3 + i0];
  p[1] = v[i1 * 3 + i1];
  p[2] = v[i1 * 3 + i2];
  p[3] = v[i2 * 3 + i1];
  p[4] = v[i2 * 3 + i2];
}

// Sliced-ELL slots, one thread per block row, for blocks other than 3x3
// (those take k_sell_slots_w33): slot k of row r takes its k-th block; the
// slot's column and source entry are written here, its values by
// k_sell_vals.
__global__ void k_sell_slots(const int64_t* rowptr, const int32_t* col,
                             int64_t nrows, const int32_t* pos,
                             const int64_t* slice_ptr, int32_t* row_len,
                             int32_t* scol, int64_t* sent) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int64_t p = pos ? (int64_t)pos[r] : r;  // position in the layout
  const int64_t s = p / kSliceH;
  const int l = (int)(p % kSliceH);
  const int64_t base = slice_ptr[s];
  const int64_t a = rowptr[r];
  const int len = (int)(rowptr[r + 1] - a);
  row_len[p] = len;
  for (int k = 0; k < len; ++k) {
    const int64_t grp = base + (int64_t)k * kSliceH;
    scol[grp + l] = col[a + k];
    sent[grp + l] = a + k;
  }
  // padding slots up to the slice's longest row get zero values and repeat
  // the row's last column (column 0 for an empty row), so a product may read
  // them unguarded: a padded term adds 0 * x[c] for a c the row already uses
  const int maxlen = (int)((slice_ptr[s + 1] - base) / kSliceH);
  const int32_t cpad = len > 0 ? col[a + len - 1] : 0;
  for (int k = len; k < maxlen; ++k) {
    scol[base + (int64_t)k * kSliceH + l] = cpad;
    sent[base + (int64_t)k * kSliceH + l] = -1;
  }
}

// Class of every 3x3 block (one thread per block, a streaming pass).
__global__ __launch_bounds__(256) void k_block_class33(
    const double* __restrict__ val, int64_t nnzb, uint8_t* __restrict__ cls) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nnzb) return;
  double v[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) v[q] = val[e * 9 + q];
  cls[e] = (uint8_t)class33(v);
}

// Sliced-ELL slots for 3x3 blocks with one wavefront per block row: lane e
// takes block e of a 64-block chunk, and the slot of a block (full blocks
// first, then the packed ones, each group in column order) is its rank
// among the row's blocks of its kind, counted with ballots.  Writes the
// slot's column with its class and its source entry, as k_sell_slots.
__global__ __launch_bounds__(256) void k_sell_slots_w33(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const uint8_t* __restrict__ bcls, int64_t nrows,
    const int64_t* __restrict__ slice_ptr, int32_t* __restrict__ row_len,
    int32_t* __restrict__ scol, int64_t* __restrict__ sent) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= nrows) return;
  const int64_t sl = r / kSliceH;
  const int l = (int)(r % kSliceH);
  const int64_t base = slice_ptr[sl];
  const int64_t a = rowptr[r];
  const int len = (int)(rowptr[r + 1] - a);
  if (lane == 0) row_len[r] = len;
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  // full blocks of the row (a second pass over the classes only for rows
  // longer than one chunk)
  int nfull = 0;
  if (len > 64)
    for (int e0 = 0; e0 < len; e0 += 64) {
      const int e = e0 + lane;
      const bool full = e < len && bcls[a + e] == 0;
      nfull += __popcll(__ballot(full));
    }
  int before_full = 0, before_packed = 0;
  for (int e0 = 0; e0 < len; e0 += 64) {
    const int e = e0 + lane;
    const int cls = e < len ? (int)bcls[a + e] : 1;
    const bool full = e < len && cls == 0;
    const bool packed = e < len && cls != 0;
    const uint64_t mf = __ballot(full), mp = __ballot(packed);
    if (len <= 64) nfull = __popcll(mf);
    if (e < len) {
      const int k = full ? before_full + __popcll(mf & lt)
                         : nfull + before_packed + __popcll(mp & lt);
      const int64_t grp = base + (int64_t)k * kSliceH;
      scol[grp + l] = (int32_t)((uint32_t)col[a + e] | ((uint32_t)cls << 30));
      sent[grp + l] = a + e;
    }
    before_full += __popcll(mf);
    before_packed += __popcll(mp);
  }
  // padding slots: packed zeros repeating the row's last column
  const int maxlen = (int)((slice_ptr[sl + 1] - base) / kSliceH);
  const int32_t cpad = (len > 0 ? col[a + len - 1] : 0) | (int32_t)(1u << 30);
  for (int k = len + lane; k < maxlen; k += 64) {
    scol[base + (int64_t)k * kSliceH + l] = cpad;
    sent[base + (int64_t)k * kSliceH + l] = -1;
  }
}

// Sliced-ELL values, one thread per slot: the slot's source block (entry
// index from the slot pass, -1 for padding and for the missing rows of a
// short last slice) is read whole and written plane by plane, so that
// consecutive threads write consecutive words of each plane.  Every value
// of the layout is written once: padding slots and the unused planes of
// packed 3x3 slots get zeros.
template <typename T, int B>
__global__ __launch_bounds__(256) void k_sell_vals(
    const int64_t* __restrict__ sent, const int32_t* __restrict__ scol,
    const double* __restrict__ val, int64_t nslots, T* __restrict__ sval) {
  static_assert((kSliceH & (kSliceH - 1)) == 0, "slice height: power of 2");
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nslots) return;
  const int64_t e = sent[i];
  const int l = (int)(i & (kSliceH - 1));
  double v[B];
#pragma unroll
  for (int q = 0; q < B; ++q) v[q] = 0.0;
  if (e >= 0) {
#pragma unroll
    for (int q = 0; q < B; ++q) v[q] = val[e * B + q];
    if constexpr (B == 9) {
      const int cls = (int)((uint32_t)scol[i] >> 30);
      if (cls) {
        double p[5];
        pack33(v, cls, p);
#pragma unroll
        for (int q = 0; q < 9; ++q) v[q] = q < 5 ? p[q] : 0.0;
      }
    }
  }
  T* dst = sval + (i - l) * B + l;
#pragma unroll
  for (int q = 0; q < B; ++q) dst[q * kSliceH] = (T)v[q];
}

__global__ void k_vrow_count(const int64_t* rowptr, int64_t nrows, int G,
                             int64_t* cnt, int32_t* row_len) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int64_t len = rowptr[r + 1] - rowptr[r];
  cnt[r] = (len + G - 1) / G;
  row_len[r] = (int32_t)len;
}

// row of every block entry
__global__ void k_entry_row(const int64_t* rowptr, int64_t nrows,
                            int32_t* row) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) row[e] = (int32_t)r;
}

// One thread per stored value: block entry e = t / B of row erow[e],
// component q = t % B.
template <typename T, int B>
__global__ void k_vrow_fill(const int64_t* rowptr, const int32_t* erow,
                            const int32_t* col, const double* val,
                            int64_t nnzb, int G, const int64_t* chunk_ptr,
                            int32_t* vcol, T* vval) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nnzb * B) return;
  const int64_t e = t / B;
  const int q = (int)(t - e * B);
  const int64_t lo = erow[e];
  const int k = (int)(e - rowptr[lo]);
  const int64_t grp = (chunk_ptr[lo] + k / G) * G;
  const int sl = k % G;
  if (q == 0) vcol[grp + sl] = col[e];
  vval[grp * B + (int64_t)q * G + sl] = (T)val[t];
}

__global__ void k_count_nz(const double* v, int64_t n,
                           unsigned long long* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long c = 0;
  for (; i < n; i += stride) c += (v[i] != 0.0);
  if (c) atomicAdd(out, c);
}

template <int BR, int BC>
void block_transpose_impl(const Bsr& a, Bsr& t, hipStream_t s,
                          TransposePlan* keep = nullptr,
                          TransposePlan* reuse = nullptr) {
  t.br = BC;
  t.bc = BR;
  t.nbr = a.nbc;
  t.nbc = a.nbr;
  t.nnzb = a.nnzb;
  if (reuse) {
    if ((int64_t)reuse->rowptr.n != t.nbr + 1 || reuse->nnzb != t.nnzb)
      throw Error(FPC_ERR_STATE, "transpose: kept plan of another shape");
    t.rowptr.alloc(t.nbr + 1);
    FPC_HIP(hipMemcpyAsync(t.rowptr.p, reuse->rowptr.p, t.rowptr.bytes(),
                           hipMemcpyDeviceToDevice, s));
    t.col.alloc(std::max<int64_t>(t.nnzb, 1));
    FPC_HIP(hipMemcpyAsync(t.col.p, reuse->col.p, t.col.bytes(),
                           hipMemcpyDeviceToDevice, s));
    t.val.alloc(std::max<int64_t>(t.nnzb * BR * BC, 1));
    if (t.nnzb)
      k_tr_gather<BR, BC><<<grid_for(t.nnzb * BR * BC, 256), 256, 0, s>>>(
          a.val.p, reuse->src.p, t.nnzb, t.val.p);
    FPC_LAUNCH_CHECK();
    if (keep) *keep = std::move(*reuse);
    return;
  }
  DevBuf<unsigned long long> cnt(a.nbc + 1);
  FPC_HIP(hipMemsetAsync(cnt.p, 0, cnt.bytes(), s));
  if (a.nbr)
    k_col_count<<<grid_for(a.nbr, 256), 256, 0, s>>>(a.rowptr.p, a.col.p,
                                                     a.nbr, cnt.p);
  FPC_LAUNCH_CHECK();
  t.rowptr.alloc(t.nbr + 1);
  scan_counts((const int64_t*)cnt.p, t.rowptr.p, t.nbr, s);
  DevBuf<unsigned long long> cursor(t.nbr + 1);
  FPC_HIP(hipMemcpyAsync(cursor.p, t.rowptr.p, (t.nbr + 1) * sizeof(int64_t),
                         hipMemcpyDeviceToDevice, s));
  t.col.alloc(std::max<int64_t>(t.nnzb, 1));
  DevBuf<int64_t> src(std::max<int64_t>(t.nnzb, 1));
  t.val.alloc(std::max<int64_t>(t.nnzb * BR * BC, 1));
  if (a.nbr)
    k_tr_fill<<<grid_for(a.nbr, 256), 256, 0, s>>>(a.rowptr.p, a.col.p, a.nbr,
                                                   cursor.p, t.col.p, src.p);
  FPC_LAUNCH_CHECK();
  if (t.nbr) {
    k_tr_sort_wave<<<(unsigned)t.nbr, 64, 0, s>>>(t.rowptr.p, t.nbr, t.col.p,
                                                  src.p);
    k_tr_sort_long<<<grid_for(t.nbr, 64), 64, 0, s>>>(t.rowptr.p, t.nbr,
                                                      t.col.p, src.p);
  }
  FPC_LAUNCH_CHECK();
  if (t.nnzb)
    k_tr_gather<BR, BC><<<grid_for(t.nnzb * BR * BC, 256), 256, 0, s>>>(
        a.val.p, src.p, t.nnzb, t.val.p);
  FPC_LAUNCH_CHECK();
  if (keep) {
    keep->nnzb = t.nnzb;
    keep->rowptr.alloc(t.nbr + 1);
    FPC_HIP(hipMemcpyAsync(keep->rowptr.p, t.rowptr.p, keep->rowptr.bytes(),
                           hipMemcpyDeviceToDevice, s));
    keep->col.alloc(std::max<int64_t>(t.nnzb, 1));
    FPC_HIP(hipMemcpyAsync(keep->col.p, t.col.p, keep->col.bytes(),
                           hipMemcpyDeviceToDevice, s));
    keep->src = std::move(src);
  }
}

template <int BR, int BC>
void to_bsr_impl(const Csr& a, Bsr& out, hipStream_t s) {
  out.br = BR;
  out.bc = BC;
  out.nbr = (a.nrows + BR - 1) / BR;
  out.nbc = (a.ncols + BC - 1) / BC;
  DevBuf<int64_t> cnt(std::max<int64_t>(out.nbr, 1));
  out.rowptr.alloc(out.nbr + 1);
  if (out.nbr) {
    k_to_bsr_w<BR, BC><<<(unsigned)out.nbr, 64, 0, s>>>(
        a.rowptr.p, a.col.p, a.val.p, a.nrows, nullptr, cnt.p, nullptr,
        nullptr);
    k_to_bsr<BR, BC><<<grid_for(out.nbr, 128), 128, 0, s>>>(
        a.rowptr.p, a.col.p, a.val.p, a.nrows, out.nbr, nullptr, cnt.p,
        nullptr, nullptr, TB_CAP);
  }
  FPC_LAUNCH_CHECK();
  out.nnzb = scan_counts_total(cnt.p, out.rowptr.p, out.nbr, s);
  out.col.alloc(std::max<int64_t>(out.nnzb, 1));
  out.val.alloc(std::max<int64_t>(out.nnzb * BR * BC, 1));
  fill_f64(out.val.p, 0.0, out.nnzb * BR * BC, s);
  if (out.nbr) {
    k_to_bsr_w<BR, BC><<<(unsigned)out.nbr, 64, 0, s>>>(
        a.rowptr.p, a.col.p, a.val.p, a.nrows, out.rowptr.p, nullptr,
        out.col.p, out.val.p);
    k_to_bsr<BR, BC><<<grid_for(out.nbr, 128), 128, 0, s>>>(
        a.rowptr.p, a.col.p, a.val.p, a.nrows, out.nbr, out.rowptr.p, nullptr,
        out.col.p, out.val.p, TB_CAP);
  }
  FPC_LAUNCH_CHECK();
}

template <int BM, int BK, int BN>
void spgemm_numeric(const Bsr& a, const Bsr& b, Bsr& c, int64_t cap,
                    int* flags, hipStream_t s, bool b_single);

template <int BM, int BK, int BN>
void spgemm_impl(const Bsr& a, const Bsr& b, Bsr& c, int* flags,
                 hipStream_t s, bool b_single, BsrPattern* keep,
                 BsrPattern* reuse) {
  c.br = BM;
  c.bc = BN;
  c.nbr = a.nbr;
  c.nbc = b.nbc;
  if (reuse) {
    if ((int64_t)reuse->rowptr.n != c.nbr + 1)
      throw Error(FPC_ERR_STATE, "spgemm: kept pattern of another shape");
    c.nnzb = reuse->nnzb;
    c.rowptr = std::move(reuse->rowptr);
    c.col = std::move(reuse->col);
    const int64_t cap = reuse->cap;
    if (keep) {
      keep->nnzb = c.nnzb;
      keep->cap = cap;
      keep->rowptr.alloc(c.nbr + 1);
      FPC_HIP(hipMemcpyAsync(keep->rowptr.p, c.rowptr.p, keep->rowptr.bytes(),
                             hipMemcpyDeviceToDevice, s));
      keep->col.alloc(std::max<int64_t>(c.nnzb, 1));
      FPC_HIP(hipMemcpyAsync(keep->col.p, c.col.p, keep->col.bytes(),
                             hipMemcpyDeviceToDevice, s));
    }
    c.val.alloc(std::max<int64_t>(c.nnzb * BM * BN, 1));
    if (c.nbr) spgemm_numeric<BM, BK, BN>(a, b, c, cap, flags, s, b_single);
    return;
  }
  DevBuf<int64_t> cnt(std::max<int64_t>(c.nbr, 1));
  DevBuf<unsigned long long> mx(2);
  c.rowptr.alloc(c.nbr + 1);
  if (!c.nbr) {
    c.nnzb = scan_counts_total(cnt.p, c.rowptr.p, 0, s);
    if (keep) {
      keep->nnzb = 0;
      keep->cap = 0;
      keep->rowptr.alloc(1);
      FPC_HIP(hipMemcpyAsync(keep->rowptr.p, c.rowptr.p, sizeof(int64_t),
                             hipMemcpyDeviceToDevice, s));
      keep->col.alloc(1);
    }
    return;
  }
  FPC_HIP(hipMemsetAsync(mx.p, 0, 2 * sizeof(unsigned long long), s));
  k_spgemm_bound<<<grid_for(c.nbr, 256), 256, 0, s>>>(a.rowptr.p, a.col.p,
                                                       b.rowptr.p, c.nbr, mx.p);
  FPC_LAUNCH_CHECK();
  unsigned long long h[2];
  FPC_HIP(hipMemcpyAsync(h, mx.p, sizeof(h), hipMemcpyDeviceToHost, s));
  FPC_HIP(hipStreamSynchronize(s));
  int bits = 6;
  while (bits < HS_MAX_BITS && (1ull << bits) < 2 * h[0]) ++bits;
  const size_t hbytes = 2 * (size_t(1) << bits) * sizeof(int);
  k_spgemm_sym<<<(unsigned)c.nbr, 64, hbytes, s>>>(
      a.rowptr.p, a.col.p, b.rowptr.p, b.col.p, c.nbr, nullptr, cnt.p, nullptr,
      flags, bits);
  FPC_LAUNCH_CHECK();
  k_max_count<<<grid_for(c.nbr, 256), 256, 0, s>>>(cnt.p, c.nbr, mx.p + 1);
  FPC_LAUNCH_CHECK();
  c.nnzb = scan_counts_total(cnt.p, c.rowptr.p, c.nbr, s);
  c.col.alloc(std::max<int64_t>(c.nnzb, 1));
  c.val.alloc(std::max<int64_t>(c.nnzb * BM * BN, 1));
  k_spgemm_sym<<<(unsigned)c.nbr, 64, hbytes, s>>>(
      a.rowptr.p, a.col.p, b.rowptr.p, b.col.p, c.nbr, c.rowptr.p, nullptr,
      c.col.p, flags, bits);
  FPC_LAUNCH_CHECK();
  FPC_HIP(hipMemcpyAsync(h, mx.p, sizeof(h), hipMemcpyDeviceToHost, s));
  FPC_HIP(hipStreamSynchronize(s));
  const int64_t cap = (int64_t)h[1];
  if (keep) {
    keep->nnzb = c.nnzb;
    keep->cap = cap;
    keep->rowptr.alloc(c.nbr + 1);
    FPC_HIP(hipMemcpyAsync(keep->rowptr.p, c.rowptr.p, keep->rowptr.bytes(),
                           hipMemcpyDeviceToDevice, s));
    keep->col.alloc(std::max<int64_t>(c.nnzb, 1));
    FPC_HIP(hipMemcpyAsync(keep->col.p, c.col.p, keep->col.bytes(),
                           hipMemcpyDeviceToDevice, s));
  }
  spgemm_numeric<BM, BK, BN>(a, b, c, cap, flags, s, b_single);
}

// The numeric phase of C = A B on C's pattern (rows of at most cap blocks).
template <int BM, int BK, int BN>
void spgemm_numeric(const Bsr& a, const Bsr& b, Bsr& c, int64_t cap,
                    int* flags, hipStream_t s, bool b_single) {
  const size_t abytes = (size_t)cap * (BM * BN * sizeof(double) + sizeof(int));
  constexpr int QM = 8;
  if (b_single && cap * BM * BN <= 64 * QM) {
    k_spgemm_num_b1<BM, BK, BN, QM><<<(unsigned)c.nbr, 64, 0, s>>>(
        a.rowptr.p, a.col.p, a.val.p, b.rowptr.p, b.col.p, b.val.p, c.nbr,
        c.rowptr.p, c.col.p, c.val.p, flags);
  } else if (abytes <= 56 * 1024) {  // with the kernel's own staging, under 64 KB
    k_spgemm_num_lds<BM, BK, BN><<<(unsigned)c.nbr, 64, abytes, s>>>(
        a.rowptr.p, a.col.p, a.val.p, b.rowptr.p, b.col.p, b.val.p, c.nbr,
        c.rowptr.p, c.col.p, c.val.p, (int)cap);
  } else {
    k_spgemm_num<BM, BK, BN><<<(unsigned)c.nbr, 64, 0, s>>>(
        a.rowptr.p, a.col.p, a.val.p, b.rowptr.p, b.col.p, b.val.p, c.nbr,
        c.rowptr.p, c.col.p, c.val.p);
  }
  FPC_LAUNCH_CHECK();
}

template <typename T, int B>
void to_sell_impl(const Bsr& a, Sell<T>& out, hipStream_t s) {
  out.br = a.br;
  out.bc = a.bc;
  out.nrows = a.nbr;
  out.nnzb = a.nnzb;
  out.nslices = (a.nbr + kSliceH - 1) / kSliceH;
  if (B == 9 && a.nbc >= (int64_t(1) << 30))
    throw Error(FPC_ERR_UNSUPPORTED, "sliced ELL: 2^30 block columns or more");
  DevBuf<int64_t> slots(std::max<int64_t>(out.nslices, 1));
  out.slice_ptr.alloc(out.nslices + 1);
  if (out.nslices)
    k_slice_len<<<grid_for(out.nslices, 128), 128, 0, s>>>(
        a.rowptr.p, nullptr, a.nbr, out.nslices, slots.p);
  FPC_LAUNCH_CHECK();
  out.nslots = scan_counts_total(slots.p, out.slice_ptr.p, out.nslices, s);
  // blocks other than 3x3 (prolongators, coarse operators, whose rows vary
  // in length): rows sorted by length within windows when that saves a
  // tenth of the slots (3x3 rows keep their order: their full and packed
  // slots line up across neighbouring rows)
  DevBuf<int32_t> pos;
  if (B != 9 && out.nslices > 1) {
    if (a.nbr >= (int64_t(1) << 31))
      throw Error(FPC_ERR_UNSUPPORTED, "sliced ELL: 2^31 block rows or more");
    DevBuf<int32_t> perm(a.nbr);
    pos.alloc(a.nbr);
    k_window_sort<<<(unsigned)((a.nbr + kSortW - 1) / kSortW), kSortT, 0, s>>>(
        a.rowptr.p, a.nbr, perm.p, pos.p);
    FPC_LAUNCH_CHECK();
    DevBuf<int64_t> sp(out.nslices + 1);
    k_slice_len<<<grid_for(out.nslices, 128), 128, 0, s>>>(
        a.rowptr.p, perm.p, a.nbr, out.nslices, slots.p);
    FPC_LAUNCH_CHECK();
    const int64_t nsort = scan_counts_total(slots.p, sp.p, out.nslices, s);
    if (10 * nsort <= 9 * out.nslots) {
      out.perm = std::move(perm);
      out.slice_ptr = std::move(sp);
      out.nslots = nsort;
    } else {
      pos.release();
    }
  }
  out.row_len.alloc(std::max<int64_t>(out.nrows, 1));
  out.col.alloc(std::max<int64_t>(out.nslots, 1));
  out.val.alloc(std::max<int64_t>(out.nslots * B, 1));
  // slots of the rows missing from a short last slice: column 0, no source
  DevBuf<int64_t> sent(std::max<int64_t>(out.nslots, 1));
  fill_i32(out.col.p, 0, out.nslots, s);
  FPC_HIP(hipMemsetAsync(sent.p, 0xff, sent.bytes(), s));
  if (out.nrows) {
    if constexpr (B == 9) {
      DevBuf<uint8_t> bcls(std::max<int64_t>(a.nnzb, 1));
      if (a.nnzb)
        k_block_class33<<<grid_for(a.nnzb, 256), 256, 0, s>>>(a.val.p, a.nnzb,
                                                              bcls.p);
      FPC_LAUNCH_CHECK();
      k_sell_slots_w33<<<(unsigned)((out.nrows + 3) / 4), 256, 0, s>>>(
          a.rowptr.p, a.col.p, bcls.p, a.nbr, out.slice_ptr.p, out.row_len.p,
          out.col.p, sent.p);
    } else
      k_sell_slots<<<grid_for(out.nrows, 256), 256, 0, s>>>(
          a.rowptr.p, a.col.p, a.nbr, pos.n ? pos.p : nullptr,
          out.slice_ptr.p, out.row_len.p, out.col.p, sent.p);
    FPC_LAUNCH_CHECK();
    k_sell_vals<T, B><<<grid_for(out.nslots, 256), 256, 0, s>>>(
        sent.p, out.col.p, a.val.p, out.nslots, out.val.p);
  }
  FPC_LAUNCH_CHECK();
}

}  // namespace

void csr_validate(const Csr& m, int* flags, hipStream_t s) {
  const double avg = m.nrows > 0 ? (double)m.nnz / (double)m.nrows : 0.0;
  const int lg = avg >= 32.0 ? 4 : avg >= 12.0 ? 3 : 2;
  k_csr_validate<<<grid_for(std::max<int64_t>(m.nrows, 1) << lg, 256), 256, 0,
                   s>>>(m.rowptr.p, m.col.p, m.val.p, m.nrows, m.ncols, m.nnz,
                        lg, flags);
  FPC_LAUNCH_CHECK();
}

void csr_active_rows(Csr& m, hipStream_t s) {
  const int64_t n = m.nrows;
  DevBuf<int64_t> f(std::max<int64_t>(n, 1)), sc(n + 1);
  if (n) {
    k_row_nonempty<<<grid_for(n, 256), 256, 0, s>>>(m.rowptr.p, n, f.p);
    FPC_LAUNCH_CHECK();
  }
  m.nact = scan_counts_total(f.p, sc.p, n, s);
  m.act.alloc(std::max<int64_t>(m.nact, 1));
  if (n) {
    k_row_list<<<grid_for(n, 256), 256, 0, s>>>(f.p, sc.p, n, m.act.p);
    FPC_LAUNCH_CHECK();
  }
}

void csr_spmv2(const Csr* m1, const double* x1, double a1, const Csr* m2,
               const double* x2, double a2, double* y, double beta,
               hipStream_t s) {
  if (m1->nrows == 0) return;
  // adding to y: only rows where m1 or m2 has a nonzero change
  if (beta == 1.0 && m1->nact >= 0 && (!m2 || m2->nact >= 0)) {
    const int64_t* rp2 = m2 ? m2->rowptr.p : nullptr;
    if (m1->nact)
      k_csr_spmv2_rows<<<grid_for(m1->nact, 256), 256, 0, s>>>(
          m1->act.p, m1->nact, 0, m1->rowptr.p, m1->col.p, m1->val.p, x1, a1,
          rp2, m2 ? m2->col.p : nullptr, m2 ? m2->val.p : nullptr, x2, a2, y,
          beta);
    if (m2 && m2->nact)
      k_csr_spmv2_rows<<<grid_for(m2->nact, 256), 256, 0, s>>>(
          m2->act.p, m2->nact, 1, m1->rowptr.p, m1->col.p, m1->val.p, x1, a1,
          rp2, m2->col.p, m2->val.p, x2, a2, y, beta);
    FPC_LAUNCH_CHECK();
    return;
  }
  k_csr_spmv2<<<grid_for(m1->nrows, 256), 256, 0, s>>>(
      m1->rowptr.p, m1->col.p, m1->val.p, x1, a1,
      m2 ? m2->rowptr.p : nullptr, m2 ? m2->col.p : nullptr,
      m2 ? m2->val.p : nullptr, x2, a2, y, beta, m1->nrows);
  FPC_LAUNCH_CHECK();
}

void csr_spmv2_many(std::initializer_list<Spmv2Call> calls, hipStream_t s) {
  Spmv2Jobs J{};
  auto add = [&](const Spmv2Call& c, const int32_t* rows, int64_t nr,
                 int skip1) {
    if (nr <= 0) return;
    if (J.n == kSpmv2Jobs) throw Error(FPC_ERR_ARG, "csr_spmv2_many: jobs");
    Spmv2Job& j = J.j[J.n];
    j.rows = rows;
    j.skip1 = skip1;
    j.rp1 = c.m1->rowptr.p;
    j.c1 = c.m1->col.p;
    j.v1 = c.m1->val.p;
    j.x1 = c.x1;
    j.a1 = c.a1;
    j.rp2 = c.m2 ? c.m2->rowptr.p : nullptr;
    j.c2 = c.m2 ? c.m2->col.p : nullptr;
    j.v2 = c.m2 ? c.m2->val.p : nullptr;
    j.x2 = c.x2;
    j.a2 = c.a2;
    j.y = c.y;
    j.beta = c.beta;
    J.start[J.n + 1] = J.start[J.n] + nr;
    ++J.n;
  };
  for (const Spmv2Call& c : calls) {
    if (c.m1->nrows == 0) continue;
    if (c.beta == 1.0 && c.m1->nact >= 0 && (!c.m2 || c.m2->nact >= 0)) {
      add(c, c.m1->act.p, c.m1->nact, 0);
      if (c.m2) add(c, c.m2->act.p, c.m2->nact, 1);
    } else {
      add(c, nullptr, c.m1->nrows, 0);
    }
  }
  if (J.n == 0) return;
  const int64_t total = J.start[J.n];
  k_csr_spmv2_multi<<<grid_for(total, 256), 256, 0, s>>>(J);
  FPC_LAUNCH_CHECK();
}

void csr_transpose(const Csr& a, Csr& t, hipStream_t s) {
  Bsr ab;
  // view the CSR as a 1x1 block matrix (arrays are borrowed, not owned)
  ab.br = ab.bc = 1;
  ab.nbr = a.nrows;
  ab.nbc = a.ncols;
  ab.nnzb = a.nnz;
  ab.rowptr.p = a.rowptr.p;
  ab.col.p = a.col.p;
  ab.val.p = a.val.p;
  Bsr tb;
  try {
    block_transpose_impl<1, 1>(ab, tb, s);
  } catch (...) {
    ab.rowptr.p = nullptr;
    ab.col.p = nullptr;
    ab.val.p = nullptr;
    throw;
  }
  ab.rowptr.p = nullptr;
  ab.col.p = nullptr;
  ab.val.p = nullptr;
  t.nrows = tb.nbr;
  t.ncols = tb.nbc;
  t.nnz = tb.nnzb;
  t.rowptr = std::move(tb.rowptr);
  t.col = std::move(tb.col);
  t.val = std::move(tb.val);
}

void csr_to_bsr(const Csr& a, int br, int bc, Bsr& out, hipStream_t s) {
  if (br == 3 && bc == 3) return to_bsr_impl<3, 3>(a, out, s);
  if (br == 3 && bc == 1) return to_bsr_impl<3, 1>(a, out, s);
  if (br == 1 && bc == 3) return to_bsr_impl<1, 3>(a, out, s);
  throw Error(FPC_ERR_ARG, "csr_to_bsr: unsupported block shape");
}

void bsr_add(const Bsr& a, const Bsr& b, Bsr& c, hipStream_t s) {
  if (a.br != b.br || a.bc != b.bc || a.nbr != b.nbr || a.nbc != b.nbc)
    throw Error(FPC_ERR_DIM, "bsr_add: shape mismatch");
  c.br = a.br;
  c.bc = a.bc;
  c.nbr = a.nbr;
  c.nbc = a.nbc;
  const int B = a.br * a.bc;
  DevBuf<int64_t> cnt(std::max<int64_t>(c.nbr, 1));
  c.rowptr.alloc(c.nbr + 1);
  if (B != 9 && B != 18 && B != 36)
    throw Error(FPC_ERR_ARG, "bsr_add: unsupported block size");
  if (c.nbr) {
    k_bsr_add_count<<<grid_for(c.nbr, 128), 128, 0, s>>>(
        a.rowptr.p, a.col.p, b.rowptr.p, b.col.p, c.nbr, cnt.p);
    FPC_LAUNCH_CHECK();
  }
  c.nnzb = scan_counts_total(cnt.p, c.rowptr.p, c.nbr, s);
  c.col.alloc(std::max<int64_t>(c.nnzb, 1));
  c.val.alloc(std::max<int64_t>(c.nnzb * B, 1));
  if (!c.nbr) return;
  const unsigned g = (unsigned)((c.nbr + 3) / 4);
  if (B == 9)
    k_bsr_add_w<9><<<g, 256, 0, s>>>(a.rowptr.p, a.col.p, a.val.p, b.rowptr.p,
                                     b.col.p, b.val.p, c.nbr, c.rowptr.p,
                                     c.col.p, c.val.p);
  else if (B == 18)
    k_bsr_add_w<18><<<g, 256, 0, s>>>(a.rowptr.p, a.col.p, a.val.p, b.rowptr.p,
                                      b.col.p, b.val.p, c.nbr, c.rowptr.p,
                                      c.col.p, c.val.p);
  else
    k_bsr_add_w<36><<<g, 256, 0, s>>>(a.rowptr.p, a.col.p, a.val.p, b.rowptr.p,
                                      b.col.p, b.val.p, c.nbr, c.rowptr.p,
                                      c.col.p, c.val.p);
  FPC_LAUNCH_CHECK();
}

void bsr_transpose(const Bsr& a, Bsr& t, hipStream_t s, TransposePlan* keep,
                   TransposePlan* reuse) {
  if (a.br == 3 && a.bc == 3)
    return block_transpose_impl<3, 3>(a, t, s, keep, reuse);
  if (a.br == 3 && a.bc == 6)
    return block_transpose_impl<3, 6>(a, t, s, keep, reuse);
  if (a.br == 6 && a.bc == 3)
    return block_transpose_impl<6, 3>(a, t, s, keep, reuse);
  if (a.br == 6 && a.bc == 6)
    return block_transpose_impl<6, 6>(a, t, s, keep, reuse);
  throw Error(FPC_ERR_ARG, "bsr_transpose: unsupported block shape");
}

void spgemm(const Bsr& a, const Bsr& b, Bsr& c, int* flags, hipStream_t s,
            bool b_single, BsrPattern* keep, BsrPattern* reuse) {
  if (a.bc != b.br || a.nbc != b.nbr)
    throw Error(FPC_ERR_DIM, "spgemm: shapes do not chain");
  const int m = a.br, k = a.bc, n = b.bc;
  if (m == 3 && k == 3 && n == 3)
    return spgemm_impl<3, 3, 3>(a, b, c, flags, s, b_single, keep, reuse);
  if (m == 3 && k == 3 && n == 6)
    return spgemm_impl<3, 3, 6>(a, b, c, flags, s, b_single, keep, reuse);
  if (m == 6 && k == 3 && n == 6)
    return spgemm_impl<6, 3, 6>(a, b, c, flags, s, b_single, keep, reuse);
  if (m == 6 && k == 6 && n == 6)
    return spgemm_impl<6, 6, 6>(a, b, c, flags, s, b_single, keep, reuse);
  if (m == 3 && k == 1 && n == 3)
    return spgemm_impl<3, 1, 3>(a, b, c, flags, s, b_single, keep, reuse);
  throw Error(FPC_ERR_ARG, "spgemm: unsupported block shapes");
}

template <typename T, int B>
void to_vrow_impl(const Bsr& a, int G, Vrow<T>& out, hipStream_t s) {
  out.br = a.br;
  out.bc = a.bc;
  out.G = G;
  out.nrows = a.nbr;
  out.nnzb = a.nnzb;
  DevBuf<int64_t> cnt(std::max<int64_t>(a.nbr, 1));
  out.chunk_ptr.alloc(a.nbr + 1);
  out.row_len.alloc(std::max<int64_t>(a.nbr, 1));
  if (a.nbr)
    k_vrow_count<<<grid_for(a.nbr, 256), 256, 0, s>>>(a.rowptr.p, a.nbr, G,
                                                      cnt.p, out.row_len.p);
  FPC_LAUNCH_CHECK();
  out.nchunks = scan_counts_total(cnt.p, out.chunk_ptr.p, a.nbr, s);
  out.col.alloc(std::max<int64_t>(out.nchunks * G, 1));
  out.val.alloc(std::max<int64_t>(out.nchunks * G * B, 1));
  fill_i32(out.col.p, 0, out.nchunks * G, s);
  FPC_HIP(hipMemsetAsync(out.val.p, 0, out.val.bytes(), s));
  if (a.nnzb) {
    DevBuf<int32_t> erow(a.nnzb);
    k_entry_row<<<grid_for(a.nbr, 256), 256, 0, s>>>(a.rowptr.p, a.nbr,
                                                     erow.p);
    k_vrow_fill<T, B><<<grid_for(a.nnzb * B, 256), 256, 0, s>>>(
        a.rowptr.p, erow.p, a.col.p, a.val.p, a.nnzb, G, out.chunk_ptr.p,
        out.col.p, out.val.p);
  }
  FPC_LAUNCH_CHECK();
}

template <typename T>
void bsr_to_vrow(const Bsr& a, int G, Vrow<T>& out, hipStream_t s) {
  const int B = a.br * a.bc;
  if (B == 9) return to_vrow_impl<T, 9>(a, G, out, s);
  if (B == 18) return to_vrow_impl<T, 18>(a, G, out, s);
  if (B == 36) return to_vrow_impl<T, 36>(a, G, out, s);
  throw Error(FPC_ERR_ARG, "bsr_to_vrow: unsupported block size");
}
template void bsr_to_vrow<double>(const Bsr&, int, Vrow<double>&, hipStream_t);
template void bsr_to_vrow<float>(const Bsr&, int, Vrow<float>&, hipStream_t);

template <typename T>
void bsr_to_sell(const Bsr& a, Sell<T>& out, hipStream_t s) {
  const int B = a.br * a.bc;
  if (B == 9) return to_sell_impl<T, 9>(a, out, s);
  if (B == 18) return to_sell_impl<T, 18>(a, out, s);
  if (B == 36) return to_sell_impl<T, 36>(a, out, s);
  throw Error(FPC_ERR_ARG, "bsr_to_sell: unsupported block size");
}
template void bsr_to_sell<double>(const Bsr&, Sell<double>&, hipStream_t);
template void bsr_to_sell<float>(const Bsr&, Sell<float>&, hipStream_t);

int64_t bsr_count_nonzeros(const Bsr& a, hipStream_t s) {
  DevBuf<unsigned long long> c(1);
  FPC_HIP(hipMemsetAsync(c.p, 0, sizeof(unsigned long long), s));
  const int64_t n = a.nnzb * a.br * a.bc;
  if (n) {
    unsigned g = grid_for(n, 256);
    if (g > 4096) g = 4096;
    k_count_nz<<<g, 256, 0, s>>>(a.val.p, n, c.p);
    FPC_LAUNCH_CHECK();
  }
  unsigned long long v = 0;
  FPC_HIP(hipMemcpyAsync(&v, c.p, sizeof(v), hipMemcpyDeviceToHost, s));
  FPC_HIP(hipStreamSynchronize(s));
  return (int64_t)v;
}

}  // namespace fpc
