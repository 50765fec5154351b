// Internal declarations of the fracprec HIP library (gfx950).
//
// Data layout on the device:
//  * Csr     scalar CSR (int64 row pointers, int32 columns, double values)
//            for the coupling blocks C1, C2, Q1, Q2, H, T.
//  * Bsr     block CSR with compile-time block shapes (3x3 node blocks on the
//            fine level, 6x6 on coarse levels, 3x6 / 6x3 transfer blocks),
//            blocks stored row-major; used by the setup (SpGEMM, transpose).
//  * Sell    sliced-ELL over block rows for the apply path: slices of 64 block
//            rows, one thread per block row, slot (slice, k, lane) holds one
//            block; the values of a (slice, k) group are component-major so a
//            wavefront loads each block component as 64 consecutive words.
#pragma once

#include <initializer_list>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "fracprec.h"

namespace fpc {

struct Error : std::runtime_error {
  fpc_status st;
  Error(fpc_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

#define FPC_HIP(x)                                                            \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess)                                                     \
      throw ::fpc::Error(e_ == hipErrorOutOfMemory ? FPC_ERR_OOM : FPC_ERR_HIP, \
                         std::string(#x) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define FPC_LAUNCH_CHECK() FPC_HIP(hipGetLastError())

// Device buffers come from the stream-ordered allocator (hipMallocAsync on
// the stream of the library call in progress, see StreamScope) through a
// block cache: a released block is kept on its (device, stream) under its
// size class and handed to the next request of that class on the same
// stream, which is safe because work on one stream runs in order.  Setups
// make hundreds of short-lived buffers; each hipFreeAsync costs tens of
// microseconds of host time, the cache none.  The cache holds at most
// kDevCacheLimit bytes (beyond that blocks go back to the pool) and is
// emptied when the last handle is destroyed or an allocation fails.
void* dev_alloc(size_t bytes, hipStream_t s, size_t* cap);
void dev_free(void* p, size_t cap, hipStream_t s);
void dev_cache_trim();
hipStream_t& alloc_stream();

struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(hipStream_t s) : prev(alloc_stream()) {
    alloc_stream() = s;
  }
  ~StreamScope() { alloc_stream() = prev; }
  StreamScope(const StreamScope&) = delete;
  StreamScope& operator=(const StreamScope&) = delete;
};

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t st = nullptr;  // stream the allocation is ordered on
  DevBuf() = default;
  explicit DevBuf(size_t n_) { alloc(n_); }
  size_t cap = 0;             // bytes of the cached block
  void alloc(size_t n_) {
    release();
    if (n_) {
      st = alloc_stream();
      p = static_cast<T*>(dev_alloc(n_ * sizeof(T), st, &cap));
      n = n_;
    }
  }
  void ensure(size_t n_) {
    if (n < n_) alloc(n_);
  }
  void release() {
    if (p) dev_free(p, cap, st);
    p = nullptr;
    n = 0;
    cap = 0;
  }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), st(o.st), cap(o.cap) {
    o.p = nullptr;
    o.n = 0;
    o.cap = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      st = o.st;
      cap = o.cap;
      o.p = nullptr;
      o.n = 0;
      o.cap = 0;
    }
    return *this;
  }
  size_t bytes() const { return n * sizeof(T); }
};

struct Csr {
  int64_t nrows = 0, ncols = 0, nnz = 0;
  DevBuf<int64_t> rowptr;
  DevBuf<int32_t> col;
  DevBuf<double> val;
  // rows holding a nonzero (ascending), when computed (nact >= 0): products
  // that add to a vector visit only these rows
  DevBuf<int32_t> act;
  int64_t nact = -1;
};

// Fill m.act / m.nact.
void csr_active_rows(Csr& m, hipStream_t s);

struct Bsr {
  int br = 0, bc = 0;
  int64_t nbr = 0, nbc = 0, nnzb = 0;
  DevBuf<int64_t> rowptr;
  DevBuf<int32_t> col;
  DevBuf<double> val;  // nnzb * br * bc, blocks row-major
};

template <typename T>
struct Sell {
  int br = 0, bc = 0;
  int64_t nrows = 0, nslices = 0, nslots = 0, nnzb = 0;
  DevBuf<int64_t> slice_ptr;  // nslices + 1, in slots (multiples of 64)
  DevBuf<int32_t> row_len;    // nrows, by position in the layout
  DevBuf<int32_t> col;        // nslots
  DevBuf<T> val;              // nslots * br * bc
  // row at each position of the layout when rows are sorted by length
  // within windows (empty: the identity)
  DevBuf<int32_t> perm;
  size_t bytes() const {
    return slice_ptr.bytes() + row_len.bytes() + col.bytes() + val.bytes() +
           perm.bytes();
  }
};

constexpr int kSliceH = 64;

// Row-group layout for operators with long rows: a group of G lanes owns one
// block row and walks it in chunks of G blocks; the values of a chunk are
// component-major (component q of the chunk's blocks is G consecutive words).
template <typename T>
struct Vrow {
  int br = 0, bc = 0, G = 0;
  int64_t nrows = 0, nchunks = 0, nnzb = 0;
  DevBuf<int64_t> chunk_ptr;  // nrows + 1, in chunks
  DevBuf<int32_t> row_len;    // nrows
  DevBuf<int32_t> col;        // nchunks * G
  DevBuf<T> val;              // nchunks * G * br * bc
  size_t bytes() const {
    return chunk_ptr.bytes() + row_len.bytes() + col.bytes() + val.bytes();
  }
};

// An apply-path operator in the layout the setup chose (by row length, or
// by timing the candidates):
// fmt 0 = sliced ELL (one thread per block row), fmt 1 = row groups; the
// batched operators use fmt 1 for one wavefront per row and fmt 2 for four.
template <typename T>
struct Op {
  int fmt = 0;
  Sell<T> s;
  Vrow<T> v;
  int64_t rows() const { return fmt ? v.nrows : s.nrows; }
  size_t bytes() const { return fmt ? v.bytes() : s.bytes(); }
};

// Device-side error flags written by validation / factorization kernels.
enum FlagIdx {
  FLAG_PATTERN = 0,
  FLAG_NAN = 1,
  FLAG_SINGULAR = 2,
  FLAG_NOT_SPD = 3,
  FLAG_OVERFLOW = 4,
  FLAG_COUNT = 8
};

// ---------------------------------------------------------------- k_util
void fill_f64(double* p, double v, int64_t n, hipStream_t s);
void fill_f32(float* p, float v, int64_t n, hipStream_t s);
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s);
// out[0] = 0, out[i+1] = sum_{j<=i} in[j]; out has n+1 entries.
void scan_counts(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);
int64_t scan_counts_total(const int64_t* in, int64_t* out, int64_t n,
                          hipStream_t s);
void i32_to_i64(const int32_t* in, int64_t* out, int64_t n, hipStream_t s);
// Deterministic two-pass reductions; results written to device memory.
void dot_f64(const double* x, const double* y, int64_t n, double* out,
             double* partials, hipStream_t s);
constexpr int kRedBlocks = 1024;
void hash32_range(uint32_t first, int64_t n, uint32_t* out, hipStream_t s);
void check_finite(const double* v, int64_t n, int* flags, hipStream_t s);
void cast_f64_f32(const double* in, float* out, int64_t n, hipStream_t s);
// True if the two CSR / block-CSR patterns (nrows + 1 row pointers, nnz
// column indices, device) are identical.
bool same_pattern(const int64_t* rp_a, const int32_t* col_a,
                  const int64_t* rp_b, const int32_t* col_b, int64_t nrows,
                  int64_t nnz, hipStream_t s);
// True if the two device arrays of n doubles are bitwise equal.
bool same_values(const double* a, const double* b, int64_t n, hipStream_t s);
void stream_triad(const double* b, const double* c, double scalar, double* a,
                  int64_t n, hipStream_t s);
double read_f64(const double* p, hipStream_t s);
int64_t read_i64(const int64_t* p, hipStream_t s);
int read_i32(const int32_t* p, hipStream_t s);

// sum over e in [b, end) of val[e] x[col[e]], added in order of e; the
// column, value and gather loads are issued four entries at a time so a
// row's gathers overlap instead of waiting one after the other.
__device__ inline double csr_row_sum(const int32_t* __restrict__ col,
                                     const double* __restrict__ val,
                                     const double* __restrict__ x, int64_t b,
                                     int64_t end) {
  double s = 0.0;
  int64_t e = b;
  for (; e + 4 <= end; e += 4) {
    const int32_t c0 = col[e], c1 = col[e + 1], c2 = col[e + 2], c3 = col[e + 3];
    const double v0 = val[e], v1 = val[e + 1], v2 = val[e + 2], v3 = val[e + 3];
    const double x0 = x[c0], x1 = x[c1], x2 = x[c2], x3 = x[c3];
    s += v0 * x0;
    s += v1 * x1;
    s += v2 * x2;
    s += v3 * x3;
  }
  for (; e < end; ++e) s += val[e] * x[col[e]];
  return s;
}

// The same on column c of KB interleaved columns (x element (j, c) at
// j KB + c).
__device__ inline double csr_row_sum_col(const int32_t* __restrict__ col,
                                         const double* __restrict__ val,
                                         const double* __restrict__ x,
                                         int64_t b, int64_t end, int KB,
                                         int c) {
  double s = 0.0;
  int64_t e = b;
  for (; e + 4 <= end; e += 4) {
    const int64_t c0 = col[e], c1 = col[e + 1], c2 = col[e + 2], c3 = col[e + 3];
    const double v0 = val[e], v1 = val[e + 1], v2 = val[e + 2], v3 = val[e + 3];
    const double x0 = x[c0 * KB + c], x1 = x[c1 * KB + c];
    const double x2 = x[c2 * KB + c], x3 = x[c3 * KB + c];
    s += v0 * x0;
    s += v1 * x1;
    s += v2 * x2;
    s += v3 * x3;
  }
  for (; e < end; ++e) s += val[e] * x[(int64_t)col[e] * KB + c];
  return s;
}

__host__ __device__ inline uint32_t lowbias32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// ---------------------------------------------------------------- k_sparse
void csr_validate(const Csr& m, int* flags, hipStream_t s);
// y = beta*y + a1*M1 x1 + a2*M2 x2 (M2 may be null); rows = M1.nrows.
void csr_spmv2(const Csr* m1, const double* x1, double a1, const Csr* m2,
               const double* x2, double a2, double* y, double beta,
               hipStream_t s);
// Several csr_spmv2 products (independent outputs, or outputs in different
// rows) in one launch, with the arithmetic of csr_spmv2 per row.
struct Spmv2Call {
  const Csr* m1;
  const double* x1;
  double a1;
  const Csr* m2;
  const double* x2;
  double a2;
  double* y;
  double beta;
};
void csr_spmv2_many(std::initializer_list<Spmv2Call> calls, hipStream_t s);
void csr_transpose(const Csr& a, Csr& t, hipStream_t s);
void csr_to_bsr(const Csr& a, int br, int bc, Bsr& out, hipStream_t s);
void bsr_add(const Bsr& a, const Bsr& b, Bsr& c, hipStream_t s);
// The pattern of a block transpose and, for each of its blocks, the source
// block, kept for a later transpose of a matrix with the same pattern.
struct TransposePlan {
  int64_t nnzb = 0;
  DevBuf<int64_t> rowptr;
  DevBuf<int32_t> col;
  DevBuf<int64_t> src;
};
// t = a^T.  reuse: the plan of an earlier transpose of the same pattern
// (only the values are gathered); keep: receives the plan.
void bsr_transpose(const Bsr& a, Bsr& t, hipStream_t s,
                   TransposePlan* keep = nullptr,
                   TransposePlan* reuse = nullptr);
// Block pattern of a product kept for a later product of operands with the
// same patterns (numeric re-setup): row pointers, block columns, and the
// longest row.
struct BsrPattern {
  int64_t nnzb = 0, cap = 0;
  DevBuf<int64_t> rowptr;
  DevBuf<int32_t> col;
};
// C = A B (block CSR; block shapes must chain).  flags[FLAG_OVERFLOW] on
// hash overflow.  b_single: every row of B holds at most one block (a
// tentative prolongator), which a faster numeric kernel uses when C's rows
// are short; a row with more raises FLAG_PATTERN.  reuse: C's pattern from
// an earlier product of operands with the same patterns (taken over; only
// the numeric phase runs); keep: receives C's pattern.
void spgemm(const Bsr& a, const Bsr& b, Bsr& c, int* flags, hipStream_t s,
            bool b_single = false, BsrPattern* keep = nullptr,
            BsrPattern* reuse = nullptr);
template <typename T>
void bsr_to_sell(const Bsr& a, Sell<T>& out, hipStream_t s);
template <typename T>
void bsr_to_vrow(const Bsr& a, int G, Vrow<T>& out, hipStream_t s);
int64_t bsr_count_nonzeros(const Bsr& a, hipStream_t s);

// ---------------------------------------------------------------- k_amg
void hinv_setup(const Csr& H, int64_t n_p, double* hinv, int* flags,
                hipStream_t s);
void bsr_block_row_scale(Bsr& b, const double* blocks3x3, hipStream_t s);
// [S_K]_k = Q2[k, K] S1[K, K]^{-1} Q1[K, k], K = nz(Q1 col k) U nz(Q2 row k)
// (eq. FS_algebraic); flags[FLAG_OVERFLOW] if |K| > 64.
void fixed_stress(const Bsr& S1, const Csr& Q1T, const Csr& Q2, double* out,
                  int* flags, hipStream_t s);
// block row i of a one-row-block BSR times alpha / M[i][i]
void bsr_row_scale_inv_diag(Bsr& b, const Csr& M, double alpha, int* flags,
                            hipStream_t s);
void bsr_dinv(const Bsr& a, double* dinv, int* flags, hipStream_t s);
// MIS-2 aggregation on the block pattern; returns n_agg, fills agg.
int64_t aggregate_mis2(const Bsr& a, int32_t* agg, DevBuf<int32_t>& roots,
                       hipStream_t s);
void rigid_modes(const double* coords, int64_t n_nodes, int nb, double* B,
                 hipStream_t s);
// Tentative prolongator per aggregate; writes ptent (n_nodes*bs*nb), Bc
// (n_agg*nb*nb), rank (n_agg).
void tentative(const int32_t* agg, int64_t n_nodes, int64_t n_agg, int bs,
               int nb, const double* B, double drop_tol, double* ptent,
               double* Bc, int32_t* rank, hipStream_t s);
void ptent_bsr(const int32_t* agg, int64_t n_nodes, int64_t n_agg, int bs,
               int nb, const double* ptent, Bsr& P, hipStream_t s);
void smooth_prolongator(Bsr& AP, const double* dinv, double omega,
                        hipStream_t s);
void dummy_diag(Bsr& Ac, const int32_t* rank, hipStream_t s);
void power_start(int64_t n_nodes, int bs, int key_stride,
                 const int32_t* node_rank, double* x, hipStream_t s);
void dense_from_bsr(const Bsr& a, int64_t npad, double* D, hipStream_t s);
// In-place inverse of an n x n (n multiple of 64) row-major matrix by
// Gauss-Jordan with partial pivoting (flags[FLAG_SINGULAR] for a column
// without a nonzero pivot candidate), or with pivot = false on the diagonal
// of an SPD matrix (flags[FLAG_NOT_SPD] for a nonpositive pivot).
void gj_inverse(double* D, int64_t n, int* flags, hipStream_t s,
                bool pivot = true);
// D (npad x npad) = [A 0; 0 I] for a row-major n x n A (device)
void dense_pad(const double* A, int64_t n, int64_t npad, double* D,
               hipStream_t s);

// ---------------------------------------------------------------- k_krylov
constexpr int kMaxKrylov = 64;
// right-hand sides of one batched solve (the widest interleaved cycle)
constexpr int kMaxBatch = 32;
// Chunk width of the row-group layout of batched operators with long rows
// (lanes per row splitting its blocks; the other 64 / 8 lanes of a
// wavefront split the columns).
constexpr int kBatchRowGroup = 8;

// ---------------------------------------------------------------- k_grad
// int32 words of work area the transmissibility gradient needs.
int64_t grad_scratch_words(int64_t n_p, int64_t n_pairs);
// Counts of every face's pairs into work[0, n_p); flags[FLAG_PATTERN] for a
// pair with an index outside [0, n_p) or K == L (skipped).
void grad_validate(int64_t n_p, int64_t n_pairs, const int32_t* pair_k,
                   const int32_t* pair_l, int32_t* work, int* flags,
                   hipStream_t s);
// After grad_validate (and a clean flag check): offsets, pair lists and the
// gradient of every face.
void grad_finish(int64_t n_p, int64_t n_pairs, const int32_t* pair_k,
                 const int32_t* pair_l, const int32_t* ndir,
                 const double* upsilon, const double* lam_p, const double* p,
                 double* grad, int32_t* work, hipStream_t s);

}  // namespace fpc
