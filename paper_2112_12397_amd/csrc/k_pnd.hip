// Pressure block S~2 (eq. app_Schur2_2; T itself without open faces or in
// t-p-u) solved exactly by a nested-dissection multifrontal factorization,
// the "nested direct solver" the paper uses for this block (Sec. 4).
//
// Ordering.  Every connected component of the face graph is bisected
// recursively by breadth-first level structures (automatic nested
// dissection): from a pseudo-peripheral face, the faces of the level that
// holds the median face separate the lower levels from the higher ones.  A
// part whose search does not reach all of it splits into the reached faces
// and the rest with an empty separator; a part of at most kNdLeaf faces is a
// leaf.  Positions: each part owns a contiguous range of the order, its two
// halves first and its separator last, so a separator is eliminated after
// everything it separates.
//
// Fronts.  Every leaf and every non-empty separator is one dense front over
// its own m faces (pivots) and the k faces of its domain's boundary (faces of
// ancestor separators adjacent to the domain).  The front is assembled from
// the separator's rows of the matrix and the children's Schur complements;
// F11 is inverted by Gauss-Jordan (in LDS up to 128 pivots, else by the
// tiled dense inverse of the coarsest AMG level; partial pivoting unless the
// block is SPD), W = F11^-1 F12 replaces F12, and F22 - F21 W (exactly
// symmetric) goes to the parent.  The first m rows then hold
// [F11^-1 | F11^-1 F12].
//
// Solve (levels of the front tree: leaves first).  Forward: b^ = b_S minus
// the contributions of descendant fronts, c_S = F11^-1 b^, contribution
// (F11^-1 F12)^T b^ to the boundary.  Backward (root first):
// x_S = c_S - F11^-1 F12 x_B.  Every output is written once, sums run in a
// fixed order, no atomics: results do not depend on scheduling.
#include <hipcub/hipcub.hpp>

#include "fpc_apply.hpp"

namespace fpc {

namespace {

constexpr int kNdT = 1024;         // threads of the ordering / factor blocks
constexpr int kNdLeaf = 128;       // largest leaf part (one level fewer than 64)
constexpr int kBndCap = 8192;      // LDS hash slots for a front's boundary
constexpr int kMaxBnd = kBndCap / 2;
constexpr int kMaxPiv = 2048;      // largest separator (pivots of one front)
constexpr int kSolveT = 1024;      // threads of the solve blocks

__device__ __forceinline__ int ld_agent(const int32_t* p) {
  return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(int32_t* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// first index a in [0, k) with B[a] >= key (B ascending)
__device__ __forceinline__ int lower_bound_i32(const int32_t* B, int k,
                                               int key) {
  int a = 0, b = k;
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (B[mid] < key) a = mid + 1;
    else b = mid;
  }
  return a;
}

// --------------------------------------------------------------- symmetry
// Every off-diagonal entry (i, j) has a partner (j, i) equal to it within a
// relative 1e-12; otherwise flags[FLAG_PATTERN].
__global__ void k_nd_symcheck(const int64_t* __restrict__ rp,
                              const int32_t* __restrict__ col,
                              const double* __restrict__ val, int64_t n,
                              int* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
    const int32_t j = col[e];
    if (j == i) continue;
    int64_t a = rp[j], b = rp[j + 1];
    while (a < b) {
      const int64_t mid = (a + b) >> 1;
      if (col[mid] < i) a = mid + 1;
      else b = mid;
    }
    if (a >= rp[j + 1] || col[a] != i) {
      atomicOr(&flags[FLAG_PATTERN], 1);
      return;
    }
    const double u = val[e], v = val[a];
    if (fabs(u - v) > 1e-12 * fmax(fabs(u), fabs(v))) {
      atomicOr(&flags[FLAG_PATTERN], 1);
      return;
    }
  }
}

// ---------------------------------------------------------------- ordering
__global__ void k_nd_label_init(int32_t* lab, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) lab[i] = (int32_t)i;
}

// one Jacobi step of min-label propagation (components get their smallest
// face as label)
__global__ void k_nd_label_prop(const int64_t* __restrict__ rp,
                                const int32_t* __restrict__ col,
                                const int32_t* __restrict__ in, int32_t* out,
                                int64_t n, int32_t* changed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t m = in[i];
  for (int64_t e = rp[i]; e < rp[i + 1]; ++e) m = min(m, in[col[e]]);
  out[i] = m;
  if (m != in[i]) atomicOr(changed, 1);
}

__global__ void k_nd_iota(int32_t* a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}

// perm sorted by component label: a component starts where the label changes
__global__ void k_nd_comp_start(const int32_t* __restrict__ lab_sorted,
                                const int32_t* __restrict__ perm, int64_t n,
                                int64_t* flag, int32_t* pos) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  flag[p] = (p == 0 || lab_sorted[p] != lab_sorted[p - 1]) ? 1 : 0;
  pos[perm[p]] = (int32_t)p;
}

// start of component c (the c-th flagged position)
__global__ void k_nd_comp_lo(const int64_t* __restrict__ flag,
                             const int64_t* __restrict__ scan, int64_t n,
                             int32_t* t_lo) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n && flag[p]) t_lo[scan[p]] = (int32_t)p;
}

// component c = part [start c, start c+1), tree node c, no parent
__global__ void k_nd_roots(int64_t n, int64_t ncomp, int4* parts,
                           const int32_t* __restrict__ t_lo, int32_t* t_hi,
                           int32_t* t_ep) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncomp) return;
  const int32_t hi = c + 1 < ncomp ? t_lo[c + 1] : (int32_t)n;
  parts[c] = make_int4(t_lo[c], hi, (int)c, 0);
  t_hi[c] = hi;
  t_ep[c] = -1;
}

// Breadth-first search over the faces whose position lies in [lo, hi), from
// face r.  Resets dist of the part's faces first; returns the number reached
// and in *last_lo the queue index where the last level starts; queue[lo ..]
// holds the reached faces level by level.  dist is accessed with agent-scope
// atomics only (the search sets it with compare-and-swap).
__device__ int nd_bfs(const int64_t* __restrict__ rp,
                      const int32_t* __restrict__ col,
                      const int32_t* __restrict__ perm,
                      const int32_t* __restrict__ pos, int lo, int hi, int r,
                      int32_t* dist, int32_t* queue, int* s_tail,
                      int* last_lo) {
  const int t = threadIdx.x;
  for (int i = lo + t; i < hi; i += kNdT) st_agent(&dist[perm[i]], -1);
  __syncthreads();
  if (t == 0) {
    st_agent(&dist[r], 0);
    queue[lo] = r;
    *s_tail = 1;
  }
  __syncthreads();
  int qa = 0, qb = 1, level = 0, lastlo = 0;
  while (qa < qb) {
    lastlo = qa;
    for (int i = qa + t; i < qb; i += kNdT) {
      const int v = queue[lo + i];
      for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
        const int u = col[e];
        const int pu = pos[u];
        if (pu < lo || pu >= hi) continue;
        if (atomicCAS(&dist[u], -1, level + 1) == -1)
          queue[lo + atomicAdd(s_tail, 1)] = u;
      }
    }
    __syncthreads();
    qa = qb;
    qb = *s_tail;
    ++level;
    __syncthreads();
  }
  *last_lo = lastlo;
  return qb;
}

// One round of the bisection: workgroup b splits parts[b] (lo, hi, node id)
// and writes its two children (lo, hi, parent, valid) to kids[2b], kids[2b+1]
// and the separator start of the node to t_slo.
__global__ __launch_bounds__(kNdT) void k_nd_split(
    const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
    const int4* __restrict__ parts, int32_t* perm, int32_t* perm2,
    int32_t* pos, int32_t* dist, int32_t* queue, int32_t* t_slo, int4* kids) {
  __shared__ int s_tail, s_min, s_cnt[3];
  __shared__ int s_wave[3][kNdT / 64];
  const int4 P = parts[blockIdx.x];
  const int lo = P.x, hi = P.y, id = P.z, size = hi - lo;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int4* kid = kids + 2 * (int64_t)blockIdx.x;
  if (size <= kNdLeaf) {
    if (t == 0) {
      t_slo[id] = lo;
      kid[0] = make_int4(0, 0, -1, 0);
      kid[1] = make_int4(0, 0, -1, 0);
    }
    return;
  }
  int lastlo;
  int reached = nd_bfs(rp, col, perm, pos, lo, hi, perm[lo], dist, queue,
                       &s_tail, &lastlo);
  int lstar = -1;
  if (reached == size) {
    // restart from the smallest face of the last level (pseudo-peripheral)
    if (t == 0) s_min = INT_MAX;
    __syncthreads();
    for (int i = lastlo + t; i < reached; i += kNdT)
      atomicMin(&s_min, queue[lo + i]);
    __syncthreads();
    const int r1 = s_min;
    reached = nd_bfs(rp, col, perm, pos, lo, hi, r1, dist, queue, &s_tail,
                     &lastlo);
    lstar = ld_agent(&dist[queue[lo + size / 2]]);
  }
  // class 0: part A (lower levels or reached), 1: separator, 2: part B
  auto cls = [&](int v) {
    const int d = ld_agent(&dist[v]);
    if (lstar < 0) return d >= 0 ? 0 : 2;
    return d < lstar ? 0 : (d == lstar ? 1 : 2);
  };
  if (t < 3) s_cnt[t] = 0;
  __syncthreads();
  for (int i = lo + t; i < hi; i += kNdT) atomicAdd(&s_cnt[cls(perm[i])], 1);
  __syncthreads();
  const int nA = s_cnt[0], nS = s_cnt[1], nB = s_cnt[2];
  int base[3] = {0, nA + nB, nA};
  // stable placement: the current order is kept inside every class
  for (int c0 = lo; c0 < hi; c0 += kNdT) {
    const int i = c0 + t;
    int c = -1, v = 0;
    if (i < hi) {
      v = perm[i];
      c = cls(v);
    }
    int my_rank = 0;
    for (int q = 0; q < 3; ++q) {
      const uint64_t b = __ballot(c == q);
      if (lane == 0) s_wave[q][wv] = __popcll(b);
      if (c == q) my_rank = __popcll(b & ((1ull << lane) - 1ull));
    }
    __syncthreads();
    if (c >= 0) {
      int before = 0;
      for (int w = 0; w < wv; ++w) before += s_wave[c][w];
      const int np = lo + base[c] + before + my_rank;
      perm2[np] = v;
      pos[v] = np;
    }
    for (int q = 0; q < 3; ++q) {
      int tot = 0;
      for (int w = 0; w < kNdT / 64; ++w) tot += s_wave[q][w];
      base[q] += tot;
    }
    __syncthreads();
  }
  for (int i = lo + t; i < hi; i += kNdT) perm[i] = perm2[i];
  if (t == 0) {
    t_slo[id] = hi - nS;
    kid[0] = nA > 0 ? make_int4(lo, lo + nA, id, 1) : make_int4(0, 0, -1, 0);
    kid[1] = nB > 0 ? make_int4(lo + nA, lo + nA + nB, id, 1)
                    : make_int4(0, 0, -1, 0);
  }
}

// Children of a round become the next round's parts, numbered from first_id
// in kid order; a child's front parent is its parent when that has a
// separator, else the parent's front parent.
__global__ __launch_bounds__(kNdT) void k_nd_compact(
    const int4* __restrict__ kids, int nk, int32_t first_id,
    const int32_t* __restrict__ t_slo, int32_t* t_lo, int32_t* t_hi,
    int32_t* t_ep, int4* parts_next, int32_t* count) {
  __shared__ int s_w[kNdT / 64];
  __shared__ int s_base;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (t == 0) s_base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < nk; c0 += kNdT) {
    const int i = c0 + t;
    const bool valid = i < nk && kids[i].w == 1;
    const uint64_t b = __ballot(valid);
    if (lane == 0) s_w[wv] = __popcll(b);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wv; ++w) before += s_w[w];
    const int rank = s_base + before + __popcll(b & ((1ull << lane) - 1ull));
    if (valid) {
      const int4 k = kids[i];
      const int id = first_id + rank;
      const int par = k.z;
      t_lo[id] = k.x;
      t_hi[id] = k.y;
      t_ep[id] = t_slo[par] < t_hi[par] ? par : t_ep[par];
      parts_next[rank] = make_int4(k.x, k.y, id, 0);
    }
    __syncthreads();
    if (t == 0) {
      int tot = 0;
      for (int w = 0; w < kNdT / 64; ++w) tot += s_w[w];
      s_base += tot;
    }
    __syncthreads();
  }
  if (t == 0) *count = s_base;
}

// ---------------------------------------------------------------- symbolic
// Heights in the front tree: nodes of one round at a time, deepest first.
__global__ void k_nd_height(int32_t a, int32_t b,
                            const int32_t* __restrict__ t_slo,
                            const int32_t* __restrict__ t_hi,
                            const int32_t* __restrict__ t_ep, int32_t* h) {
  const int32_t id = a + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (id >= b) return;
  if (t_slo[id] < t_hi[id] && t_ep[id] >= 0)
    atomicMax(&h[t_ep[id]], h[id] + 1);
}

// sort key of a node: its height for fronts, H for empty separators
__global__ void k_nd_front_key(int32_t nn, const int32_t* __restrict__ t_slo,
                               const int32_t* __restrict__ t_hi,
                               const int32_t* __restrict__ h, int32_t H,
                               int32_t* key, int32_t* lev_cnt) {
  const int32_t id = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (id >= nn) return;
  const bool front = t_slo[id] < t_hi[id];
  key[id] = front ? h[id] : H;
  if (front) atomicAdd(&lev_cnt[h[id]], 1);
}

__global__ void k_nd_front_fields(
    int32_t nf, const int32_t* __restrict__ ids,
    const int32_t* __restrict__ t_lo, const int32_t* __restrict__ t_hi,
    const int32_t* __restrict__ t_slo, int32_t* fidx, int32_t* f_lo,
    int32_t* f_slo, int32_t* f_m) {
  const int32_t f = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (f >= nf) return;
  const int32_t id = ids[f];
  fidx[id] = f;
  f_lo[f] = t_lo[id];
  f_slo[f] = t_slo[id];
  f_m[f] = t_hi[id] - t_slo[id];
}

// front parent (front index, -1 for roots) as sort key + 1, children counts
__global__ void k_nd_front_parent(int32_t nf, const int32_t* __restrict__ ids,
                                  const int32_t* __restrict__ t_ep,
                                  const int32_t* __restrict__ fidx,
                                  int32_t* pkey, int64_t* pcnt) {
  const int32_t f = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (f >= nf) return;
  const int32_t ep = t_ep[ids[f]];
  const int32_t k = ep >= 0 ? fidx[ep] + 1 : 0;
  pkey[f] = k;
  atomicAdd((unsigned long long*)&pcnt[k], 1ull);
}

// Boundary of front f: positions >= hi adjacent to its domain [lo, hi),
// collected in an LDS hash set.  With f_bnd == nullptr only the count is
// written (f_k); otherwise the sorted list goes to bnd + f_bnd[f].
__global__ __launch_bounds__(kNdT) void k_nd_bnd(
    const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ pos,
    const int32_t* __restrict__ f_lo, const int32_t* __restrict__ f_slo,
    const int32_t* __restrict__ f_m, int32_t* f_k,
    const int64_t* __restrict__ f_bnd, int32_t* bnd, int* flags) {
  __shared__ int32_t tab[kBndCap];
  __shared__ int32_t lst[kMaxBnd];
  __shared__ int s_n, s_over;
  const int f = blockIdx.x, t = threadIdx.x;
  const int lo = f_lo[f], hi = f_slo[f] + f_m[f];
  for (int i = t; i < kBndCap; i += kNdT) tab[i] = -1;
  if (t == 0) {
    s_n = 0;
    s_over = 0;
  }
  __syncthreads();
  for (int i = lo + t; i < hi; i += kNdT) {
    const int v = perm[i];
    for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
      const int pu = pos[col[e]];
      if (pu < lo) {
        atomicOr(&flags[FLAG_PATTERN], 1);  // not a nested dissection
        continue;
      }
      if (pu < hi) continue;
      uint32_t hs = ((uint32_t)pu * 2654435761u) & (kBndCap - 1);
      int probe = 0;
      for (; probe < kBndCap; ++probe) {
        const int old = atomicCAS(&tab[hs], -1, pu);
        if (old == -1) {
          atomicAdd(&s_n, 1);
          break;
        }
        if (old == pu) break;
        hs = (hs + 1) & (kBndCap - 1);
      }
      if (probe == kBndCap) s_over = 1;
    }
  }
  __syncthreads();
  const int k = s_n;
  if (s_over || k > kMaxBnd) {
    if (t == 0) {
      atomicOr(&flags[FLAG_OVERFLOW], 1);
      f_k[f] = 0;
    }
    return;
  }
  if (!f_bnd) {
    if (t == 0) f_k[f] = k;
    return;
  }
  // compact, pad to a power of two, bitonic sort
  if (t == 0) s_n = 0;
  __syncthreads();
  for (int i = t; i < kBndCap; i += kNdT)
    if (tab[i] >= 0) lst[atomicAdd(&s_n, 1)] = tab[i];
  int np2 = 1;
  while (np2 < k) np2 <<= 1;
  __syncthreads();
  for (int i = k + t; i < np2; i += kNdT) lst[i] = INT_MAX;
  __syncthreads();
  for (int size = 2; size <= np2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = t; i < np2 / 2; i += kNdT) {
        const int a = 2 * i - (i & (stride - 1));
        const int b = a + stride;
        const bool up = (a & size) == 0;
        const int x = lst[a], y = lst[b];
        if ((x > y) == up) {
          lst[a] = y;
          lst[b] = x;
        }
      }
      __syncthreads();
    }
  }
  int32_t* out = bnd + f_bnd[f];
  for (int i = t; i < k; i += kNdT) out[i] = lst[i];
}

__global__ void k_nd_sizes(int32_t nf, const int32_t* __restrict__ f_m,
                           const int32_t* __restrict__ f_k, int64_t* kcnt,
                           int64_t* fcnt) {
  const int32_t f = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (f >= nf) return;
  const int64_t ld = (int64_t)f_m[f] + f_k[f];
  kcnt[f] = f_k[f];
  fcnt[f] = ld * ld;
}

__global__ void k_nd_slot_keys(int64_t ns, const int32_t* __restrict__ bnd,
                               int32_t* key, int32_t* slot, int64_t* gcnt) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ns) return;
  key[q] = bnd[q];
  slot[q] = (int32_t)q;
  atomicAdd((unsigned long long*)&gcnt[bnd[q]], 1ull);
}

// ---------------------------------------------------------------- numeric
// Block reduction of (|value|, index): largest value, smallest index on
// ties.  All threads return the winner.
__device__ void nd_argmax(double v, int idx, double* s_v, int* s_i,
                          double* out_v, int* out_i) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o);
    const int oi = __shfl_xor(idx, o);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  if (lane == 0) {
    s_v[wv] = v;
    s_i[wv] = idx;
  }
  __syncthreads();
  if (t == 0) {
    double bv = s_v[0];
    int bi = s_i[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      if (s_v[w] > bv || (s_v[w] == bv && s_i[w] < bi)) {
        bv = s_v[w];
        bi = s_i[w];
      }
    s_v[0] = bv;
    s_i[0] = bi;
  }
  __syncthreads();
  *out_v = s_v[0];
  *out_i = s_i[0];
  __syncthreads();
}

// Assembly of the fronts [f0, f0 + gridDim.x) of one level: the separator's
// rows of the matrix (sk, nullable, subtracted from the diagonal: S~2 = T -
// S_K) with their mirror into F21, then the children's Schur complements,
// one child after the other (deterministic).
__global__ __launch_bounds__(kNdT) void k_nd_assemble(
    int32_t f0, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ sk,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ pos,
    const int32_t* __restrict__ f_slo, const int32_t* __restrict__ f_m,
    const int32_t* __restrict__ f_k, const int64_t* __restrict__ f_F,
    const int64_t* __restrict__ f_bnd, const int32_t* __restrict__ bnd,
    const int64_t* __restrict__ ch_off, const int32_t* __restrict__ ch,
    double* F, int* flags) {
  __shared__ int s_map[kMaxBnd];
  const int f = f0 + blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = kNdT / 64;
  const int m = f_m[f], k = f_k[f], ld = m + k, slo = f_slo[f], hi = slo + m;
  double* __restrict__ A = F + f_F[f];
  const int32_t* __restrict__ B = bnd + f_bnd[f];
  for (int64_t i = t; i < (int64_t)ld * ld; i += kNdT) A[i] = 0.0;
  __syncthreads();
  // the separator's rows of the matrix (and their mirror into F21)
  for (int r = t; r < m; r += kNdT) {
    const int v = perm[slo + r];
    for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
      const int pu = pos[col[e]];
      if (pu < slo) continue;
      int c;
      if (pu < hi) {
        c = pu - slo;
      } else {
        const int a = lower_bound_i32(B, k, pu);
        if (a >= k || B[a] != pu) {
          atomicOr(&flags[FLAG_PATTERN], 1);
          continue;
        }
        c = m + a;
      }
      A[(int64_t)r * ld + c] = val[e];
      if (c >= m) A[(int64_t)c * ld + r] = val[e];
    }
    if (sk) A[(int64_t)r * ld + r] -= sk[v];
  }
  __syncthreads();
  // children's Schur complements, one child after the other
  for (int64_t ci = ch_off[f + 1]; ci < ch_off[f + 2]; ++ci) {
    const int c = ch[ci];
    const int mc = f_m[c], kc = f_k[c], ldc = mc + kc;
    const double* __restrict__ U = F + f_F[c] + (int64_t)mc * ldc + mc;
    const int32_t* __restrict__ Bc = bnd + f_bnd[c];
    for (int a = t; a < kc; a += kNdT) {
      const int p = Bc[a];
      int idx = -1;
      if (p >= slo && p < hi) {
        idx = p - slo;
      } else if (p >= hi) {
        const int q = lower_bound_i32(B, k, p);
        if (q < k && B[q] == p) idx = m + q;
      }
      if (idx < 0) atomicOr(&flags[FLAG_PATTERN], 1);
      s_map[a] = idx;
    }
    __syncthreads();
    for (int a = wv; a < kc; a += nw) {
      const int ra = s_map[a];
      if (ra < 0) continue;
      for (int b = lane; b < kc; b += 64) {
        const int cb = s_map[b];
        if (cb >= 0) A[(int64_t)ra * ld + cb] += U[(int64_t)a * ldc + b];
      }
    }
    __syncthreads();
  }
}

// F11 <- F11^-1 in LDS for fronts with at most kLdsPiv pivots (list fl):
// Gauss-Jordan, pivots on the diagonal when spd (a nonpositive one flags
// FLAG_NOT_SPD), partial pivoting otherwise (a pivot at or below 1e-14 of
// the block's largest entry flags FLAG_SINGULAR).
constexpr int kLdsPiv = 128;
static_assert(kNdLeaf <= kLdsPiv, "leaf fronts are inverted in LDS");
__global__ __launch_bounds__(kNdT) void k_nd_inv_lds(
    const int32_t* __restrict__ fl, const int32_t* __restrict__ f_m,
    const int32_t* __restrict__ f_k, const int64_t* __restrict__ f_F,
    double* F, int spd, int* flags) {
  __shared__ double S[kLdsPiv * kLdsPiv];
  __shared__ double s_col[kLdsPiv];
  __shared__ int s_piv[kLdsPiv];
  __shared__ double s_rv[kNdT / 64];
  __shared__ int s_ri[kNdT / 64];
  const int f = fl[blockIdx.x];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = kNdT / 64;
  const int m = f_m[f], ld = m + f_k[f];
  double* __restrict__ A = F + f_F[f];
  double vmax = 0.0;
  for (int i = wv; i < m; i += nw)
    for (int j = lane; j < m; j += 64) {
      const double x = A[(int64_t)i * ld + j];
      S[i * m + j] = x;
      vmax = fmax(vmax, fabs(x));
    }
  double amax, dv;
  int di;
  nd_argmax(vmax, 0, s_rv, s_ri, &amax, &di);
  for (int kk = 0; kk < m; ++kk) {
    int p = kk;
    if (!spd) {
      double bv = -1.0;
      int bi = kk;
      for (int i = kk + t; i < m; i += kNdT) {
        const double x = fabs(S[i * m + kk]);
        if (x > bv) {
          bv = x;
          bi = i;
        }
      }
      nd_argmax(bv, bi, s_rv, s_ri, &dv, &p);
      if (p != kk) {
        for (int j = t; j < m; j += kNdT) {
          const double x = S[kk * m + j];
          S[kk * m + j] = S[p * m + j];
          S[p * m + j] = x;
        }
        __syncthreads();
      }
    }
    if (t == 0) s_piv[kk] = p;
    for (int i = t; i < m; i += kNdT) s_col[i] = S[i * m + kk];
    __syncthreads();
    const double d = s_col[kk];
    const bool bad = spd ? !(d > 0.0) || !isfinite(d)
                         : !(fabs(d) > 1e-14 * amax) || !isfinite(d);
    if (bad) {
      if (t == 0) atomicOr(&flags[spd ? FLAG_NOT_SPD : FLAG_SINGULAR], 1);
      return;  // uniform: every thread read the same pivot
    }
    const double inv = 1.0 / d;
    for (int j = t; j < m; j += kNdT)
      S[kk * m + j] = (j == kk ? 1.0 : S[kk * m + j]) * inv;
    __syncthreads();
    for (int i = wv; i < m; i += nw) {
      const double fi = s_col[i];
      if (i == kk || fi == 0.0) continue;
      for (int j = lane; j < m; j += 64)
        S[i * m + j] = (j == kk ? 0.0 : S[i * m + j]) - fi * S[kk * m + j];
    }
    __syncthreads();
  }
  if (!spd)
    for (int kk = m - 1; kk >= 0; --kk) {
      const int p = s_piv[kk];
      if (p == kk) continue;
      for (int i = t; i < m; i += kNdT) {
        const double x = S[i * m + kk];
        S[i * m + kk] = S[i * m + p];
        S[i * m + p] = x;
      }
      __syncthreads();
    }
  for (int i = wv; i < m; i += nw)
    for (int j = lane; j < m; j += 64) A[(int64_t)i * ld + j] = S[i * m + j];
}

// [F11 0; 0 I] (npad x npad) from a front, and F11^-1 back
__global__ void k_nd_pad(const double* __restrict__ A, int ld, int m,
                         int npad, double* __restrict__ P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)npad * npad) return;
  const int i = (int)(idx / npad), j = (int)(idx % npad);
  P[idx] = (i < m && j < m) ? A[(int64_t)i * ld + j] : (i == j ? 1.0 : 0.0);
}
__global__ void k_nd_unpad(const double* __restrict__ P, int npad, int m,
                           double* __restrict__ A, int ld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int i = (int)(idx / m), j = (int)(idx % m);
  A[(int64_t)i * ld + j] = P[(int64_t)i * npad + j];
}

// 64 x 64 output tiles of the two front products, 256 threads with 4 x 4
// outputs each, the inner dimension (the m pivots) in chunks of 16 through
// LDS.  Item (f, ti, tj):
//   kind 0: W = F11^-1 F12 into the F12 block, F12 read as the transpose of
//           F21 (the two are assembled as exact mirrors);
//   kind 1: F22 <- F22 - F21 W, tiles with ti <= tj only, each value written
//           to both (a, b) and (b, a), so the complement passed to the parent
//           is exactly symmetric.
constexpr int kTile = 64, kTk = 16;
template <int KIND>
__global__ __launch_bounds__(256) void k_nd_tile(
    const int4* __restrict__ items, const int32_t* __restrict__ f_m,
    const int32_t* __restrict__ f_k, const int64_t* __restrict__ f_F,
    double* F) {
  __shared__ double As[kTk][kTile + 1];
  __shared__ double Bs[kTk][kTile + 1];
  const int4 it = items[blockIdx.x];
  const int f = it.x, ti = it.y, tj = it.z;
  const int m = f_m[f], k = f_k[f], ld = m + k;
  double* __restrict__ A = F + f_F[f];
  const int rows = KIND == 0 ? m : k;   // output rows
  const int cols = k;                   // output columns
  const int r0 = ti * kTile, c0 = tj * kTile;
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int j0 = 0; j0 < m; j0 += kTk) {
    // A tile: rows r0.., inner j0..; B tile: inner j0.., columns c0..
    for (int e = t; e < kTile * kTk; e += 256) {
      const int r = e / kTk, q = e % kTk;
      const int gr = r0 + r, gj = j0 + q;
      double av = 0.0, bv = 0.0;
      if (gr < rows && gj < m)
        av = KIND == 0 ? A[(int64_t)gr * ld + gj]            // F11^-1
                       : A[(int64_t)(m + gr) * ld + gj];     // F21
      const int gc = c0 + r;
      if (gc < cols && gj < m)
        bv = KIND == 0 ? A[(int64_t)(m + gc) * ld + gj]      // F12^T = F21
                       : A[(int64_t)gj * ld + m + gc];       // W
      As[q][r] = av;
      Bs[q][r] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kTk; ++q) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[q][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[q][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gr = r0 + ty + 16 * i, gc = c0 + tx + 16 * j;
      if (gr >= rows || gc >= cols) continue;
      if (KIND == 0) {
        A[(int64_t)gr * ld + m + gc] = acc[i][j];
      } else {
        if (ti == tj && gr > gc) continue;
        const double u = A[(int64_t)(m + gr) * ld + m + gc] - acc[i][j];
        A[(int64_t)(m + gr) * ld + m + gc] = u;
        A[(int64_t)(m + gc) * ld + m + gr] = u;
      }
    }
}

// ------------------------------------------------------------------ solve
// Forward step of one level, single column.  Item (f, c0): outputs
// c0 .. c0 + 63 of [c_S ; y_B] = [F11^-1 | F11^-1 F12]^T b^ of front f,
// 16 groups of 64 threads splitting the pivots.
__global__ __launch_bounds__(kSolveT) void k_nd_fwd(
    const int2* __restrict__ items, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ f_slo, const int32_t* __restrict__ f_m,
    const int32_t* __restrict__ f_k, const int64_t* __restrict__ f_F,
    const int64_t* __restrict__ f_bnd, const int64_t* __restrict__ g_off,
    const int32_t* __restrict__ g_slot, const double* __restrict__ F,
    const double* __restrict__ in, double* __restrict__ xp,
    double* __restrict__ contrib, double* __restrict__ out) {
  __shared__ double s_b[kMaxPiv];
  __shared__ double s_part[kSolveT / 64][64];
  const int2 it = items[blockIdx.x];
  const int f = it.x, c0 = it.y;
  const int t = threadIdx.x, lane = t & 63, g = t >> 6;
  const int m = f_m[f], k = f_k[f], ld = m + k, slo = f_slo[f];
  for (int j = t; j < m; j += kSolveT) {
    const int p = slo + j;
    double v = in[perm[p]];
    for (int64_t q = g_off[p]; q < g_off[p + 1]; ++q) v -= contrib[g_slot[q]];
    s_b[j] = v;
  }
  __syncthreads();
  const int c = c0 + lane;
  const double* __restrict__ M = F + f_F[f];
  double acc = 0.0;
  if (c < ld)
    for (int j = g; j < m; j += kSolveT / 64)
      acc += M[(int64_t)j * ld + c] * s_b[j];
  s_part[g][lane] = acc;
  __syncthreads();
  if (t < 64 && c < ld) {
    double sum = 0.0;
    for (int q = 0; q < kSolveT / 64; ++q) sum += s_part[q][lane];
    if (c < m) {
      xp[slo + c] = sum;
      if (k == 0) out[perm[slo + c]] = sum;
    } else {
      contrib[f_bnd[f] + (c - m)] = sum;
    }
  }
}

// Backward step of one level, single column.  Item (f, j0): rows
// j0 .. j0 + 15 of x_S = c_S - (F11^-1 F12) x_B, a wavefront per row.
__global__ __launch_bounds__(kSolveT) void k_nd_bwd(
    const int2* __restrict__ items, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ f_slo, const int32_t* __restrict__ f_m,
    const int32_t* __restrict__ f_k, const int64_t* __restrict__ f_F,
    const int64_t* __restrict__ f_bnd, const int32_t* __restrict__ bnd,
    const double* __restrict__ F, double* __restrict__ xp,
    double* __restrict__ out) {
  __shared__ double s_x[kMaxBnd];
  const int2 it = items[blockIdx.x];
  const int f = it.x, j0 = it.y;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m = f_m[f], k = f_k[f], ld = m + k, slo = f_slo[f];
  const int32_t* __restrict__ B = bnd + f_bnd[f];
  for (int a = t; a < k; a += kSolveT) s_x[a] = xp[B[a]];
  __syncthreads();
  const int j = j0 + w;
  if (j >= m) return;
  const double* __restrict__ row = F + f_F[f] + (int64_t)j * ld + m;
  double acc = 0.0;
  for (int a = lane; a < k; a += 64) acc += row[a] * s_x[a];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) {
    const double v = xp[slo + j] - acc;
    xp[slo + j] = v;
    out[perm[slo + j]] = v;
  }
}

// The same two steps on KB interleaved columns (element (i, c) at i KB + c),
// with the single-column kernels' summation order, so that every column
// equals a single-column solve bit for bit.
__global__ __launch_bounds__(kSolveT) void k_nd_fwd_b(
    const int2* __restrict__ items, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ f_slo, const int32_t* __restrict__ f_m,
    const int32_t* __restrict__ f_k, const int64_t* __restrict__ f_F,
    const int64_t* __restrict__ f_bnd, const int64_t* __restrict__ g_off,
    const int32_t* __restrict__ g_slot, const double* __restrict__ F,
    const double* __restrict__ in, double* __restrict__ bp,
    double* __restrict__ xp, double* __restrict__ contrib,
    double* __restrict__ out, int KB) {
  const int2 it = items[blockIdx.x];
  const int f = it.x, c0 = it.y;
  const int t = threadIdx.x;
  const int m = f_m[f], k = f_k[f], ld = m + k, slo = f_slo[f];
  // every item of the front gathers b^ (identical values)
  for (int idx = t; idx < m * KB; idx += kSolveT) {
    const int j = idx / KB, cc = idx - j * KB;
    const int p = slo + j;
    double v = in[(int64_t)perm[p] * KB + cc];
    for (int64_t q = g_off[p]; q < g_off[p + 1]; ++q)
      v -= contrib[(int64_t)g_slot[q] * KB + cc];
    bp[(int64_t)p * KB + cc] = v;
  }
  __syncthreads();
  const double* __restrict__ M = F + f_F[f];
  constexpr int G = kSolveT / 64;  // pivot groups of the single-column kernel
  for (int oc = t; oc < 64 * KB; oc += kSolveT) {
    const int c = c0 + oc / KB, cc = oc % KB;
    if (c >= ld) continue;
    double sum = 0.0;
    for (int g = 0; g < G; ++g) {
      double acc = 0.0;
      for (int j = g; j < m; j += G)
        acc += M[(int64_t)j * ld + c] * bp[(int64_t)(slo + j) * KB + cc];
      sum += acc;
    }
    if (c < m) {
      xp[(int64_t)(slo + c) * KB + cc] = sum;
      if (k == 0) out[(int64_t)perm[slo + c] * KB + cc] = sum;
    } else {
      contrib[(f_bnd[f] + (c - m)) * KB + cc] = sum;
    }
  }
}

// a wavefront per (row, column), lanes over the boundary as in k_nd_bwd
__global__ __launch_bounds__(kSolveT) void k_nd_bwd_b(
    const int2* __restrict__ items, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ f_slo, const int32_t* __restrict__ f_m,
    const int32_t* __restrict__ f_k, const int64_t* __restrict__ f_F,
    const int64_t* __restrict__ f_bnd, const int32_t* __restrict__ bnd,
    const double* __restrict__ F, double* __restrict__ xp,
    double* __restrict__ out, int KB) {
  const int2 it = items[blockIdx.x];
  const int f = it.x, j0 = it.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = f_m[f], k = f_k[f], ld = m + k, slo = f_slo[f];
  const int32_t* __restrict__ B = bnd + f_bnd[f];
  const int nrow = min(16, m - j0);
  for (int pr = w; pr < nrow * KB; pr += kSolveT / 64) {
    const int j = j0 + pr / KB, cc = pr % KB;
    const double* __restrict__ row = F + f_F[f] + (int64_t)j * ld + m;
    double acc = 0.0;
    for (int a = lane; a < k; a += 64)
      acc += row[a] * xp[(int64_t)B[a] * KB + cc];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) {
      const double v = xp[(int64_t)(slo + j) * KB + cc] - acc;
      xp[(int64_t)(slo + j) * KB + cc] = v;
      out[(int64_t)perm[slo + j] * KB + cc] = v;
    }
  }
}

// ------------------------------------------------------------------- host
void sort_pairs(const int32_t* kin, int32_t* kout, const int32_t* vin,
                int32_t* vout, int64_t n, int end_bit, hipStream_t s) {
  if (n <= 0) return;
  size_t bytes = 0;
  FPC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, kin, kout, vin,
                                             vout, (int)n, 0, end_bit, s));
  DevBuf<char> tmp(std::max<size_t>(bytes, 1));
  FPC_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, bytes, kin, kout, vin,
                                             vout, (int)n, 0, end_bit, s));
}

int bits_for(int64_t v) {
  int b = 1;
  while (b < 31 && (int64_t(1) << b) <= v) ++b;
  return b;
}

template <typename T>
std::vector<T> to_host(const T* d, int64_t n, hipStream_t s) {
  std::vector<T> h(std::max<int64_t>(n, 0));
  if (n > 0)
    FPC_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost,
                           s));
  FPC_HIP(hipStreamSynchronize(s));
  return h;
}

template <typename T>
void to_device(DevBuf<T>& d, const std::vector<T>& h, hipStream_t s) {
  d.alloc(std::max<size_t>(h.size(), 1));
  if (!h.empty())
    FPC_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T),
                           hipMemcpyHostToDevice, s));
}

// Ordering and symbolic analysis (pattern only).
void nd_analyse(PSolve& ps, const Csr& T, int* flags, hipStream_t s) {
  const int64_t n = T.nrows;
  if (n >= INT32_MAX / 4)
    throw Error(FPC_ERR_UNSUPPORTED, "pressure block: too many faces");
  const unsigned g = grid_for(n, 256);
  // connected components (min-label propagation), faces grouped by
  // component in increasing order
  DevBuf<int32_t> la(n), lb(n), changed(1);
  k_nd_label_init<<<g, 256, 0, s>>>(la.p, n);
  FPC_LAUNCH_CHECK();
  for (int64_t it = 0;; it += 8) {
    fill_i32(changed.p, 0, 1, s);
    for (int q = 0; q < 8; ++q) {
      k_nd_label_prop<<<g, 256, 0, s>>>(T.rowptr.p, T.col.p, la.p, lb.p, n,
                                        changed.p);
      std::swap(la, lb);
    }
    FPC_LAUNCH_CHECK();
    if (read_i32(changed.p, s) == 0) break;
    if (it > 4 * n + 8) throw Error(FPC_ERR_HIP, "component labelling stalled");
  }
  ps.perm.alloc(n);
  ps.pos.alloc(n);
  DevBuf<int32_t> iota(n), lsorted(n);
  k_nd_iota<<<g, 256, 0, s>>>(iota.p, n);
  FPC_LAUNCH_CHECK();
  sort_pairs(la.p, lsorted.p, iota.p, ps.perm.p, n, bits_for(n), s);
  DevBuf<int64_t> flag(n), scan(n + 1);
  k_nd_comp_start<<<g, 256, 0, s>>>(lsorted.p, ps.perm.p, n, flag.p, ps.pos.p);
  FPC_LAUNCH_CHECK();
  const int64_t ncomp = scan_counts_total(flag.p, scan.p, n, s);
  // tree nodes: at most one per face and one per empty separator
  const int64_t cap = 3 * n + 4;
  DevBuf<int32_t> t_lo(cap), t_hi(cap), t_slo(cap), t_ep(cap);
  DevBuf<int4> parts_a(n), parts_b(n), kids(2 * n);
  DevBuf<int32_t> perm2(n), dist(n), queue(n), count(1);
  k_nd_comp_lo<<<g, 256, 0, s>>>(flag.p, scan.p, n, t_lo.p);
  FPC_LAUNCH_CHECK();
  k_nd_roots<<<grid_for(ncomp, 256), 256, 0, s>>>(n, ncomp, parts_a.p, t_lo.p,
                                                  t_hi.p, t_ep.p);
  FPC_LAUNCH_CHECK();
  std::vector<int32_t> round_first{0};
  int32_t n_nodes = (int32_t)ncomp, cnt = (int32_t)ncomp;
  while (cnt > 0) {
    if ((int64_t)round_first.size() > n + 2)
      throw Error(FPC_ERR_HIP, "nested dissection: bisection did not finish");
    k_nd_split<<<cnt, kNdT, 0, s>>>(T.rowptr.p, T.col.p, parts_a.p, ps.perm.p,
                                    perm2.p, ps.pos.p, dist.p, queue.p,
                                    t_slo.p, kids.p);
    FPC_LAUNCH_CHECK();
    k_nd_compact<<<1, kNdT, 0, s>>>(kids.p, 2 * cnt, n_nodes, t_slo.p, t_lo.p,
                                    t_hi.p, t_ep.p, parts_b.p, count.p);
    FPC_LAUNCH_CHECK();
    const int32_t nxt = read_i32(count.p, s);
    round_first.push_back(n_nodes);
    n_nodes += nxt;
    if (n_nodes > cap) throw Error(FPC_ERR_HIP, "nested dissection: tree overflow");
    cnt = nxt;
    std::swap(parts_a, parts_b);
  }
  round_first.push_back(n_nodes);
  // heights in the front tree, deepest round first
  DevBuf<int32_t> h(n_nodes);
  fill_i32(h.p, 0, n_nodes, s);
  for (int r = (int)round_first.size() - 2; r >= 1; --r) {
    const int32_t a = round_first[r], b = round_first[r + 1];
    if (b > a)
      k_nd_height<<<grid_for(b - a, 256), 256, 0, s>>>(a, b, t_slo.p, t_hi.p,
                                                       t_ep.p, h.p);
  }
  FPC_LAUNCH_CHECK();
  // the number of levels: heights are below the number of rounds
  const int32_t Hcap = (int32_t)round_first.size();
  DevBuf<int32_t> key(n_nodes), keys(n_nodes), ids_all(n_nodes), lev_cnt(Hcap + 1);
  fill_i32(lev_cnt.p, 0, Hcap + 1, s);
  k_nd_front_key<<<grid_for(n_nodes, 256), 256, 0, s>>>(
      n_nodes, t_slo.p, t_hi.p, h.p, Hcap, key.p, lev_cnt.p);
  FPC_LAUNCH_CHECK();
  DevBuf<int32_t> iota2(n_nodes);
  k_nd_iota<<<grid_for(n_nodes, 256), 256, 0, s>>>(iota2.p, n_nodes);
  FPC_LAUNCH_CHECK();
  sort_pairs(key.p, keys.p, iota2.p, ids_all.p, n_nodes, bits_for(Hcap), s);
  std::vector<int32_t> lc = to_host(lev_cnt.p, Hcap, s);
  ps.lev_off.assign(1, 0);
  for (int l = 0; l < Hcap && lc[l] > 0; ++l)
    ps.lev_off.push_back(ps.lev_off.back() + lc[l]);
  ps.n_levels = (int)ps.lev_off.size() - 1;
  const int32_t nf = (int32_t)ps.lev_off.back();
  ps.n_fronts = nf;
  // per-front fields
  DevBuf<int32_t> fidx(n_nodes), f_lo(nf);
  ps.f_slo.alloc(nf);
  ps.f_m.alloc(nf);
  ps.f_k.alloc(nf);
  k_nd_front_fields<<<grid_for(nf, 256), 256, 0, s>>>(
      nf, ids_all.p, t_lo.p, t_hi.p, t_slo.p, fidx.p, f_lo.p, ps.f_slo.p,
      ps.f_m.p);
  FPC_LAUNCH_CHECK();
  // children lists: fronts sorted by front parent (stable: ascending front)
  DevBuf<int32_t> pkey(nf), pkeys(nf), fi(nf);
  DevBuf<int64_t> pcnt(nf + 1);
  fill_i64(pcnt.p, 0, nf + 1, s);
  k_nd_front_parent<<<grid_for(nf, 256), 256, 0, s>>>(nf, ids_all.p, t_ep.p,
                                                      fidx.p, pkey.p, pcnt.p);
  FPC_LAUNCH_CHECK();
  k_nd_iota<<<grid_for(nf, 256), 256, 0, s>>>(fi.p, nf);
  FPC_LAUNCH_CHECK();
  ps.ch.alloc(nf);
  ps.ch_off.alloc(nf + 2);
  sort_pairs(pkey.p, pkeys.p, fi.p, ps.ch.p, nf, bits_for(nf + 1), s);
  scan_counts(pcnt.p, ps.ch_off.p, nf + 1, s);
  // boundaries: sizes, offsets, sorted lists
  k_nd_bnd<<<nf, kNdT, 0, s>>>(T.rowptr.p, T.col.p, ps.perm.p, ps.pos.p, f_lo.p,
                               ps.f_slo.p, ps.f_m.p, ps.f_k.p, nullptr, nullptr,
                               flags);
  FPC_LAUNCH_CHECK();
  DevBuf<int64_t> kcnt(nf), fcnt(nf);
  k_nd_sizes<<<grid_for(nf, 256), 256, 0, s>>>(nf, ps.f_m.p, ps.f_k.p, kcnt.p,
                                               fcnt.p);
  FPC_LAUNCH_CHECK();
  ps.f_bnd.alloc(nf + 1);
  ps.f_F.alloc(nf + 1);
  ps.n_slots = scan_counts_total(kcnt.p, ps.f_bnd.p, nf, s);
  ps.F_words = scan_counts_total(fcnt.p, ps.f_F.p, nf, s);
  ps.bnd.alloc(std::max<int64_t>(ps.n_slots, 1));
  k_nd_bnd<<<nf, kNdT, 0, s>>>(T.rowptr.p, T.col.p, ps.perm.p, ps.pos.p, f_lo.p,
                               ps.f_slo.p, ps.f_m.p, ps.f_k.p, ps.f_bnd.p,
                               ps.bnd.p, flags);
  FPC_LAUNCH_CHECK();
  // contribution gather lists: slots grouped by target position
  ps.g_off.alloc(n + 1);
  ps.g_slot.alloc(std::max<int64_t>(ps.n_slots, 1));
  {
    DevBuf<int64_t> gcnt(n);
    fill_i64(gcnt.p, 0, n, s);
    const int64_t ns = ps.n_slots;
    if (ns > 0) {
      DevBuf<int32_t> sk_(ns), skeys(ns), sl(ns);
      k_nd_slot_keys<<<grid_for(ns, 256), 256, 0, s>>>(ns, ps.bnd.p, sk_.p,
                                                       sl.p, gcnt.p);
      FPC_LAUNCH_CHECK();
      sort_pairs(sk_.p, skeys.p, sl.p, ps.g_slot.p, ns, bits_for(n), s);
    }
    scan_counts(gcnt.p, ps.g_off.p, n, s);
  }
  // host copies of the front sizes: work lists of the solve, size checks
  ps.hm = to_host(ps.f_m.p, nf, s);
  ps.hk = to_host(ps.f_k.p, nf, s);
  for (int32_t f = 0; f < nf; ++f)
    if (ps.hm[f] > kMaxPiv)
      throw Error(FPC_ERR_UNSUPPORTED,
                  "pressure block: a separator of more than 2048 faces");
  std::vector<int2> fw, bw;
  ps.fwd_off.assign(1, 0);
  ps.bwd_off.assign(1, 0);
  for (int l = 0; l < ps.n_levels; ++l) {
    for (int64_t f = ps.lev_off[l]; f < ps.lev_off[l + 1]; ++f) {
      const int m = ps.hm[f], k = ps.hk[f];
      for (int c0 = 0; c0 < m + k; c0 += 64) fw.push_back(make_int2((int)f, c0));
      if (k > 0)
        for (int j0 = 0; j0 < m; j0 += 16) bw.push_back(make_int2((int)f, j0));
    }
    ps.fwd_off.push_back((int64_t)fw.size());
    ps.bwd_off.push_back((int64_t)bw.size());
  }
  to_device(ps.fwd_items, fw, s);
  to_device(ps.bwd_items, bw, s);
  // numeric phase: fronts whose F11 is inverted in LDS, the larger ones (by
  // the tiled dense Gauss-Jordan), the 64 x 64 tiles of W and of the Schur
  // complements; host offsets of the front matrices
  std::vector<int32_t> sm;
  std::vector<int4> wt, st;
  ps.small_off.assign(1, 0);
  ps.w_off.assign(1, 0);
  ps.s_off.assign(1, 0);
  ps.big.assign(ps.n_levels, {});
  ps.hF.assign(nf + 1, 0);
  for (int32_t f = 0; f < nf; ++f) {
    const int64_t ld = (int64_t)ps.hm[f] + ps.hk[f];
    ps.hF[f + 1] = ps.hF[f] + ld * ld;
  }
  for (int l = 0; l < ps.n_levels; ++l) {
    for (int64_t f = ps.lev_off[l]; f < ps.lev_off[l + 1]; ++f) {
      const int m = ps.hm[f], k = ps.hk[f];
      if (m <= kLdsPiv) sm.push_back((int32_t)f);
      else ps.big[l].push_back((int32_t)f);
      const int tm = (m + kTile - 1) / kTile, tk = (k + kTile - 1) / kTile;
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tk; ++b) wt.push_back(make_int4((int)f, a, b, 0));
      for (int a = 0; a < tk; ++a)
        for (int b = a; b < tk; ++b) st.push_back(make_int4((int)f, a, b, 0));
    }
    ps.small_off.push_back((int64_t)sm.size());
    ps.w_off.push_back((int64_t)wt.size());
    ps.s_off.push_back((int64_t)st.size());
  }
  to_device(ps.small, sm, s);
  to_device(ps.w_items, wt, s);
  to_device(ps.s_items, st, s);
  ps.xp.alloc(n);
  ps.contrib.alloc(std::max<int64_t>(ps.n_slots, 1));
  ps.n = n;
  FPC_HIP(hipStreamSynchronize(s));
}

}  // namespace

// Factor (values) for the current analysis, level by level: assembly,
// F11^-1, W = F11^-1 F12, Schur complements for the parents.
void psolve_factor(PSolve& ps, const Csr& T, const double* sk, bool spd,
                   int* flags, hipStream_t s) {
  ps.spd = spd;
  ps.F.alloc(std::max<int64_t>(ps.F_words, 1));
  DevBuf<double> pad;
  for (int l = 0; l < ps.n_levels; ++l) {
    const int64_t a = ps.lev_off[l], b = ps.lev_off[l + 1];
    if (b == a) continue;
    k_nd_assemble<<<(unsigned)(b - a), kNdT, 0, s>>>(
        (int32_t)a, T.rowptr.p, T.col.p, T.val.p, sk, ps.perm.p, ps.pos.p,
        ps.f_slo.p, ps.f_m.p, ps.f_k.p, ps.f_F.p, ps.f_bnd.p, ps.bnd.p,
        ps.ch_off.p, ps.ch.p, ps.F.p, flags);
    FPC_LAUNCH_CHECK();
    const int64_t sa = ps.small_off[l], sb = ps.small_off[l + 1];
    if (sb > sa)
      k_nd_inv_lds<<<(unsigned)(sb - sa), kNdT, 0, s>>>(
          ps.small.p + sa, ps.f_m.p, ps.f_k.p, ps.f_F.p, ps.F.p, spd ? 1 : 0,
          flags);
    FPC_LAUNCH_CHECK();
    for (int32_t f : ps.big[l]) {
      const int m = ps.hm[f], ld = m + ps.hk[f];
      const int npad = (int)((m + 63) / 64 * 64);
      pad.ensure((size_t)npad * npad);
      double* A = ps.F.p + ps.hF[f];
      k_nd_pad<<<grid_for((int64_t)npad * npad, 256), 256, 0, s>>>(A, ld, m,
                                                                  npad, pad.p);
      FPC_LAUNCH_CHECK();
      gj_inverse(pad.p, npad, flags, s, /*pivot=*/!spd);
      k_nd_unpad<<<grid_for((int64_t)m * m, 256), 256, 0, s>>>(pad.p, npad, m,
                                                              A, ld);
      FPC_LAUNCH_CHECK();
    }
    const int64_t wa = ps.w_off[l], wb = ps.w_off[l + 1];
    if (wb > wa)
      k_nd_tile<0><<<(unsigned)(wb - wa), 256, 0, s>>>(
          ps.w_items.p + wa, ps.f_m.p, ps.f_k.p, ps.f_F.p, ps.F.p);
    const int64_t ta = ps.s_off[l], tb = ps.s_off[l + 1];
    if (tb > ta)
      k_nd_tile<1><<<(unsigned)(tb - ta), 256, 0, s>>>(
          ps.s_items.p + ta, ps.f_m.p, ps.f_k.p, ps.f_F.p, ps.F.p);
    FPC_LAUNCH_CHECK();
  }
}

void psolve_analyse(PSolve& ps, const Csr& T, int* flags, hipStream_t s) {
  ps = PSolve();
  if (T.nrows == 0) return;
  k_nd_symcheck<<<grid_for(T.nrows, 256), 256, 0, s>>>(
      T.rowptr.p, T.col.p, T.val.p, T.nrows, flags);
  FPC_LAUNCH_CHECK();
  nd_analyse(ps, T, flags, s);
}

int64_t psolve_factor_entries(const PSolve& ps) {
  int64_t e = 0;
  for (int64_t f = 0; f < ps.n_fronts; ++f)
    e += (int64_t)ps.hm[f] * (ps.hm[f] + ps.hk[f]);
  return e;
}

int64_t psolve_solve_bytes(const PSolve& ps) {
  int64_t fwd = 0, bwd = 0;
  for (int64_t f = 0; f < ps.n_fronts; ++f) {
    fwd += (int64_t)ps.hm[f] * (ps.hm[f] + ps.hk[f]);
    bwd += (int64_t)ps.hm[f] * ps.hk[f];
  }
  return 8 * (fwd + bwd) + ps.n * (12 + 12 + 16) + ps.n_slots * (16 + 4 + 4);
}

void psolve_apply(const PSolve& ps, const double* in, double* out,
                  int64_t n_p, int trans, hipStream_t s) {
  (void)trans;  // the operator is symmetric
  if (!n_p) return;
  for (int l = 0; l < ps.n_levels; ++l) {
    const int64_t a = ps.fwd_off[l], b = ps.fwd_off[l + 1];
    if (b > a)
      k_nd_fwd<<<(unsigned)(b - a), kSolveT, 0, s>>>(
          ps.fwd_items.p + a, ps.perm.p, ps.f_slo.p, ps.f_m.p, ps.f_k.p,
          ps.f_F.p, ps.f_bnd.p, ps.g_off.p, ps.g_slot.p, ps.F.p, in, ps.xp.p,
          ps.contrib.p, out);
  }
  for (int l = ps.n_levels - 2; l >= 0; --l) {
    const int64_t a = ps.bwd_off[l], b = ps.bwd_off[l + 1];
    if (b > a)
      k_nd_bwd<<<(unsigned)(b - a), kSolveT, 0, s>>>(
          ps.bwd_items.p + a, ps.perm.p, ps.f_slo.p, ps.f_m.p, ps.f_k.p,
          ps.f_F.p, ps.f_bnd.p, ps.bnd.p, ps.F.p, ps.xp.p, out);
  }
  FPC_LAUNCH_CHECK();
}

void psolve_batch_buffers(PSolve& ps, int KB) {
  if (ps.KB == KB) return;
  ps.KB = KB;
  ps.bpB.alloc(std::max<int64_t>(ps.n, 1) * KB);
  ps.xpB.alloc(std::max<int64_t>(ps.n, 1) * KB);
  ps.contribB.alloc(std::max<int64_t>(ps.n_slots, 1) * KB);
}

void psolve_apply_b(const PSolve& ps, const double* in, double* out,
                    int64_t n_p, int KB, hipStream_t s) {
  if (!n_p) return;
  if (ps.KB != KB)
    throw Error(FPC_ERR_STATE, "pressure solve: batch buffers not sized");
  for (int l = 0; l < ps.n_levels; ++l) {
    const int64_t a = ps.fwd_off[l], b = ps.fwd_off[l + 1];
    if (b > a)
      k_nd_fwd_b<<<(unsigned)(b - a), kSolveT, 0, s>>>(
          ps.fwd_items.p + a, ps.perm.p, ps.f_slo.p, ps.f_m.p, ps.f_k.p,
          ps.f_F.p, ps.f_bnd.p, ps.g_off.p, ps.g_slot.p, ps.F.p, in, ps.bpB.p,
          ps.xpB.p, ps.contribB.p, out, KB);
  }
  for (int l = ps.n_levels - 2; l >= 0; --l) {
    const int64_t a = ps.bwd_off[l], b = ps.bwd_off[l + 1];
    if (b > a)
      k_nd_bwd_b<<<(unsigned)(b - a), kSolveT, 0, s>>>(
          ps.bwd_items.p + a, ps.perm.p, ps.f_slo.p, ps.f_m.p, ps.f_k.p,
          ps.f_F.p, ps.f_bnd.p, ps.bnd.p, ps.F.p, ps.xpB.p, out, KB);
  }
  FPC_LAUNCH_CHECK();
}

}  // namespace fpc
