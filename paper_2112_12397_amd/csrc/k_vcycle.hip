// Apply path: sliced-ELL block SpMV with fused Chebyshev epilogues, the
// V-cycle driver, the coarsest dense solve, the exact pressure-block solve
// and the small kernels of the block preconditioner (Alg 3.2 / 3.4).
#include "fpc_apply.hpp"

namespace fpc {

namespace {

// Workgroups are dispatched round-robin over the 8 XCDs of MI355X; remap so
// that every XCD walks a contiguous range of slices (neighbouring rows share
// x entries in that XCD's L2).
__device__ inline int64_t xcd_block(int64_t b, int64_t G) {
  const int64_t q = G >> 3, r = G & 7;
  const int64_t x = b & 7, w = b >> 3;
  return x * q + (x < r ? x : r) + w;
}

template <typename T>
struct SellView {
  int64_t nrows, nslices;
  const int64_t* __restrict__ slice_ptr;
  const int32_t* __restrict__ row_len;
  const int32_t* __restrict__ col;
  const T* __restrict__ val;
};

template <typename T>
SellView<T> view(const Sell<T>& a) {
  return SellView<T>{a.nrows, a.nslices, a.slice_ptr.p, a.row_len.p,
                     a.col.p, a.val.p};
}

// ---------------------------------------------------------------- loaders
template <typename T, int NV>
struct LoadX {
  const T* __restrict__ x;
  __device__ T operator()(int64_t dof, int v) const { return x[dof * NV + v]; }
};

// first Chebyshev direction d0 = D^{-1} b / theta, formed on the fly
template <typename T, int NV>
struct LoadScaled {
  const T* __restrict__ b;
  const T* __restrict__ dinv;
  T inv_theta;
  __device__ T operator()(int64_t dof, int v) const {
    return dinv[dof] * b[dof * NV + v] * inv_theta;
  }
};

// ---------------------------------------------------------------- epilogues
template <typename T, int BR, int NV>
struct EpiStore {
  T* __restrict__ y;
  __device__ void operator()(int64_t row, int v, const T* acc) const {
#pragma unroll
    for (int i = 0; i < BR; ++i) y[(row * BR + i) * NV + v] = acc[i];
  }
};

template <typename T, int BR, int NV>
struct EpiAdd {
  T* __restrict__ y;
  __device__ void operator()(int64_t row, int v, const T* acc) const {
#pragma unroll
    for (int i = 0; i < BR; ++i) y[(row * BR + i) * NV + v] += acc[i];
  }
};

template <typename T, int BR>
struct EpiDinv {
  const T* __restrict__ dinv;
  T* __restrict__ y;
  __device__ void operator()(int64_t row, int v, const T* acc) const {
#pragma unroll
    for (int i = 0; i < BR; ++i) y[row * BR + i] = dinv[row * BR + i] * acc[i];
  }
};

// Pre-smoothing from x = 0, two Chebyshev steps fused around q = A d0:
//   R1 = b - q, r1 = D^-1 R1, d1 = c1 d0 + c2 r1, x = d0 + d1.
template <typename T, int BR, int NV>
struct EpiPre1 {
  const T* __restrict__ b;
  const T* __restrict__ dinv;
  T* __restrict__ x;
  T* __restrict__ d;
  T* __restrict__ R;
  T inv_theta, c1, c2;
  __device__ void operator()(int64_t row, int v, const T* acc) const {
#pragma unroll
    for (int i = 0; i < BR; ++i) {
      const int64_t dof = row * BR + i, k = dof * NV + v;
      const T bi = b[k], di = dinv[dof];
      const T d0 = di * bi * inv_theta;
      const T R1 = bi - acc[i];
      const T r1 = di * R1;
      const T d1 = c1 * d0 + c2 * r1;
      x[k] = d0 + d1;
      d[k] = d1;
      R[k] = R1;
    }
  }
};

// residual after pre-smoothing: res = R1 - A d1 = b - A x
template <typename T, int BR, int NV>
struct EpiRes {
  const T* __restrict__ R;
  T* __restrict__ res;
  __device__ void operator()(int64_t row, int v, const T* acc) const {
#pragma unroll
    for (int i = 0; i < BR; ++i) {
      const int64_t k = (row * BR + i) * NV + v;
      res[k] = R[k] - acc[i];
    }
  }
};

// post-smoothing step 1 around q = A x: r0 = D^-1 (b - q), d0 = r0 / theta,
// xo = x + d0
template <typename T, int BR, int NV>
struct EpiPost1 {
  const T* __restrict__ b;
  const T* __restrict__ dinv;
  const T* __restrict__ xin;
  T* __restrict__ xo;
  T* __restrict__ d;
  T* __restrict__ r;
  T inv_theta;
  __device__ void operator()(int64_t row, int v, const T* acc) const {
#pragma unroll
    for (int i = 0; i < BR; ++i) {
      const int64_t dof = row * BR + i, k = dof * NV + v;
      const T r0 = dinv[dof] * (b[k] - acc[i]);
      const T d0 = r0 * inv_theta;
      xo[k] = xin[k] + d0;
      d[k] = d0;
      r[k] = r0;
    }
  }
};

// post-smoothing step 2 around q = A d0: r1 = r0 - D^-1 q,
// d1 = c1 d0 + c2 r1, xo += d1
template <typename T, int BR, int NV>
struct EpiPost2 {
  const T* __restrict__ dinv;
  const T* __restrict__ r;
  const T* __restrict__ din;
  T* __restrict__ xo;
  T c1, c2;
  __device__ void operator()(int64_t row, int v, const T* acc) const {
#pragma unroll
    for (int i = 0; i < BR; ++i) {
      const int64_t dof = row * BR + i, k = dof * NV + v;
      const T r1 = r[k] - dinv[dof] * acc[i];
      xo[k] += c1 * din[k] + c2 * r1;
    }
  }
};

// ---------------------------------------------------------------- SpMV
// One thread per (block row, column); a wavefront covers 64/NV consecutive
// block rows of one 64-row slice, so the block components of a slot group
// are read as contiguous 64-wide vectors.
template <typename T, int BR, int BC, int NV, class Load, class Epi>
__global__ __launch_bounds__(256) void k_sell(SellView<T> A, Load ld,
                                              Epi epi) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t gw = blk * 4 + wave;
  const int64_t slice = gw / NV;
  if (slice >= A.nslices) return;
  const int sub = (int)(gw % NV);
  const int rloc = sub * (64 / NV) + lane / NV;
  const int v = lane % NV;
  const int64_t row = slice * kSliceH + rloc;
  if (row >= A.nrows) return;
  const int len = A.row_len[row];
  const int64_t base = A.slice_ptr[slice];
  const int32_t* __restrict__ cp = A.col + base + rloc;
  const T* __restrict__ vp = A.val + base * (BR * BC) + rloc;
  T acc[BR];
#pragma unroll
  for (int i = 0; i < BR; ++i) acc[i] = T(0);
#pragma unroll 2
  for (int k = 0; k < len; ++k) {
    const int64_t c = cp[(int64_t)k * kSliceH];
    const T* __restrict__ vb = vp + (int64_t)k * kSliceH * (BR * BC);
    T xv[BC];
#pragma unroll
    for (int j = 0; j < BC; ++j) xv[j] = ld(c * BC + j, v);
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int j = 0; j < BC; ++j) acc[i] += vb[(i * BC + j) * kSliceH] * xv[j];
  }
  epi(row, v, acc);
}

template <typename T, int BR, int BC, int NV, class Load, class Epi>
void launch_sell(const Sell<T>& A, Load ld, Epi epi, hipStream_t s) {
  if (A.nrows == 0) return;
  const int64_t waves = A.nslices * NV;
  const unsigned grid = (unsigned)((waves + 3) / 4);
  k_sell<T, BR, BC, NV, Load, Epi><<<grid, 256, 0, s>>>(view(A), ld, epi);
  FPC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- coarsest
// x = Ainv b on the coarsest level (FP64 arithmetic), one wavefront per row.
template <typename T, int NV>
__global__ __launch_bounds__(256) void k_coarse(const double* __restrict__ Ai,
                                                int64_t ld, int64_t n,
                                                const T* __restrict__ b,
                                                T* __restrict__ x) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  const double* __restrict__ a = Ai + row * ld;
  for (int64_t k = lane; k < n; k += 64) {
    const double m = a[k];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += m * (double)b[k * NV + v];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v)
    for (int off = 32; off > 0; off >>= 1) acc[v] += __shfl_xor(acc[v], off, 64);
  if (lane < NV) {
    double out = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (v == lane) out = acc[v];
    x[row * NV + lane] = (T)out;
  }
}

// ---------------------------------------------------------------- interface
__global__ void k_face_apply(const double* __restrict__ hinv,
                             const double* __restrict__ in,
                             double* __restrict__ out, int64_t n_p, int trans) {
  int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= n_p) return;
  const double* h = hinv + K * 9;
  const double a = in[3 * K], b = in[3 * K + 1], c = in[3 * K + 2];
  if (!trans) {
    out[3 * K] = h[0] * a + h[1] * b + h[2] * c;
    out[3 * K + 1] = h[3] * a + h[4] * b + h[5] * c;
    out[3 * K + 2] = h[6] * a + h[7] * b + h[8] * c;
  } else {
    out[3 * K] = h[0] * a + h[3] * b + h[6] * c;
    out[3 * K + 1] = h[1] * a + h[4] * b + h[7] * c;
    out[3 * K + 2] = h[2] * a + h[5] * b + h[8] * c;
  }
}

// out[i*nv + col] = (T)(base_i + a1 (M1 x1)_i + a2 (M2 x2)_i)
template <typename T>
__global__ void k_to_level(T* __restrict__ out, int nv, int colv,
                           const double* __restrict__ base,
                           const int64_t* rp1, const int32_t* c1,
                           const double* v1, const double* x1, double a1,
                           const int64_t* rp2, const int32_t* c2,
                           const double* v2, const double* x2, double a2,
                           int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double r = base ? base[i] : 0.0;
  if (rp1) {
    double s = 0.0;
    for (int64_t e = rp1[i]; e < rp1[i + 1]; ++e) s += v1[e] * x1[c1[e]];
    r += a1 * s;
  }
  if (rp2) {
    double s = 0.0;
    for (int64_t e = rp2[i]; e < rp2[i + 1]; ++e) s += v2[e] * x2[c2[e]];
    r += a2 * s;
  }
  out[i * nv + colv] = (T)r;
}

template <typename T>
__global__ void k_from_level(const T* __restrict__ xo, int nv, int64_t n,
                             double* __restrict__ vu, int diff) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  vu[i] = diff ? (double)xo[i * nv] - (double)xo[i * nv + 1] : (double)xo[i * nv];
}

// v_t = -t_t + H~^{-1} (C v_u) face by face (Alg 3.4 steps 9-10)
__global__ void k_tface(const int64_t* __restrict__ rp,
                        const int32_t* __restrict__ col,
                        const double* __restrict__ val,
                        const double* __restrict__ vu,
                        const double* __restrict__ t_t,
                        const double* __restrict__ hinv,
                        double* __restrict__ v_t, int64_t n_p, int trans) {
  int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= n_p) return;
  double s[3];
  for (int r = 0; r < 3; ++r) {
    double a = 0.0;
    const int64_t row = 3 * K + r;
    for (int64_t e = rp[row]; e < rp[row + 1]; ++e) a += val[e] * vu[col[e]];
    s[r] = a;
  }
  const double* h = hinv + K * 9;
  for (int r = 0; r < 3; ++r) {
    double hv = trans ? h[0 * 3 + r] * s[0] + h[1 * 3 + r] * s[1] + h[2 * 3 + r] * s[2]
                      : h[r * 3 + 0] * s[0] + h[r * 3 + 1] * s[1] + h[r * 3 + 2] * s[2];
    v_t[3 * K + r] = -t_t[3 * K + r] + hv;
  }
}

// exact pressure-block solve: one wavefront per (component, row)
__global__ __launch_bounds__(256) void k_psolve(
    const double* __restrict__ dense, const int64_t* __restrict__ dense_off,
    const int64_t* __restrict__ comp_off, const int64_t* __restrict__ comp_pad,
    const int32_t* __restrict__ comp_of_row, const int32_t* __restrict__ members,
    const double* __restrict__ in, double* __restrict__ out, int64_t n_p,
    int trans) {
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= n_p) return;
  const int c = comp_of_row[g];
  const int64_t o = comp_off[c];
  const int64_t n = comp_off[c + 1] - o;
  const int64_t ld = comp_pad[c];
  const int64_t r = g - o;
  const double* M = dense + dense_off[c];
  double acc = 0.0;
  if (!trans)
    for (int64_t k = lane; k < n; k += 64) acc += M[r * ld + k] * in[members[o + k]];
  else
    for (int64_t k = lane; k < n; k += 64) acc += M[k * ld + r] * in[members[o + k]];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) out[members[g]] = acc;
}

template <typename T, int NV>
__global__ void k_zero(T* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * NV) p[i] = T(0);
}

// ---------------------------------------------------------------- V-cycle
template <typename T>
const Sell<T>& selA(const Level& L, bool tr);
template <>
const Sell<double>& selA<double>(const Level& L, bool tr) {
  return tr ? L.sAT : L.sA;
}
template <>
const Sell<float>& selA<float>(const Level& L, bool tr) {
  return tr ? L.fAT : L.fA;
}
template <typename T>
const Sell<T>& selP(const Level& L);
template <>
const Sell<double>& selP<double>(const Level& L) { return L.sP; }
template <>
const Sell<float>& selP<float>(const Level& L) { return L.fP; }
template <typename T>
const Sell<T>& selR(const Level& L);
template <>
const Sell<double>& selR<double>(const Level& L) { return L.sR; }
template <>
const Sell<float>& selR<float>(const Level& L) { return L.fR; }
template <typename T>
const T* seldinv(const Level& L);
template <>
const double* seldinv<double>(const Level& L) { return L.dinv.p; }
template <>
const float* seldinv<float>(const Level& L) { return L.dinv32.p; }

template <typename T, int BS, int NV>
void smooth_level(const Level& L, LevelVecs<T>& v, bool tr, hipStream_t s,
                  int phase, KTimer* timer) {
  const Sell<T>& A = selA<T>(L, tr);
  const T* dinv = seldinv<T>(L);
  const T it = T(1.0 / L.theta), c1 = T(L.c1), c2 = T(L.c2);
  if (phase == 0) {
    launch_sell<T, BS, BS, NV>(A, LoadScaled<T, NV>{v.b.p, dinv, it},
                               EpiPre1<T, BS, NV>{v.b.p, dinv, v.x.p, v.d.p,
                                                  v.r.p, it, c1, c2},
                               s);
    if (timer) timer->begin(s);
    launch_sell<T, BS, BS, NV>(A, LoadX<T, NV>{v.d.p},
                               EpiRes<T, BS, NV>{v.r.p, v.res.p}, s);
    if (timer) timer->end(s);
  } else {
    launch_sell<T, BS, BS, NV>(A, LoadX<T, NV>{v.x.p},
                               EpiPost1<T, BS, NV>{v.b.p, dinv, v.x.p, v.xo.p,
                                                   v.d.p, v.r.p, it},
                               s);
    launch_sell<T, BS, BS, NV>(A, LoadX<T, NV>{v.d.p},
                               EpiPost2<T, BS, NV>{dinv, v.r.p, v.d.p, v.xo.p,
                                                   c1, c2},
                               s);
  }
}

template <typename T, int BS, int NB, int NV>
void restrict_level(const Level& L, LevelVecs<T>& v, LevelVecs<T>& vc,
                    hipStream_t s) {
  launch_sell<T, NB, BS, NV>(selR<T>(L), LoadX<T, NV>{v.res.p},
                             EpiStore<T, NB, NV>{vc.b.p}, s);
}

template <typename T, int BS, int NB, int NV>
void prolong_level(const Level& L, LevelVecs<T>& v, LevelVecs<T>& vc,
                   hipStream_t s) {
  launch_sell<T, BS, NB, NV>(selP<T>(L), LoadX<T, NV>{vc.xo.p},
                             EpiAdd<T, BS, NV>{v.x.p}, s);
}

template <typename T, int NV>
void dispatch_smooth(const Level& L, LevelVecs<T>& v, bool tr, hipStream_t s,
                     int phase, KTimer* timer) {
  if (L.bs == 3) smooth_level<T, 3, NV>(L, v, tr, s, phase, timer);
  else smooth_level<T, 6, NV>(L, v, tr, s, phase, timer);
}

template <typename T, int NV>
void dispatch_transfer(const Level& L, LevelVecs<T>& v, LevelVecs<T>& vc,
                       hipStream_t s, bool restr) {
  if (L.bs == 3 && L.nb == 6) {
    if (restr) restrict_level<T, 3, 6, NV>(L, v, vc, s);
    else prolong_level<T, 3, 6, NV>(L, v, vc, s);
  } else if (L.bs == 3 && L.nb == 3) {
    if (restr) restrict_level<T, 3, 3, NV>(L, v, vc, s);
    else prolong_level<T, 3, 3, NV>(L, v, vc, s);
  } else {
    if (restr) restrict_level<T, 6, 6, NV>(L, v, vc, s);
    else prolong_level<T, 6, 6, NV>(L, v, vc, s);
  }
}

template <typename T, int NV>
void vcycle_rec(Hierarchy& H, CycleVecs<T>& cv, size_t l, bool tr,
                hipStream_t s) {
  const Level& L = H.L[l];
  LevelVecs<T>& v = cv.lv[l];
  if (L.coarsest) {
    const double* Ai = tr ? H.AinvT.p : H.Ainv.p;
    const unsigned g = (unsigned)((H.nc + 3) / 4);
    k_coarse<T, NV><<<g, 256, 0, s>>>(Ai, H.ncpad, H.nc, v.b.p, v.xo.p);
    FPC_LAUNCH_CHECK();
    return;
  }
  KTimer* timer = (l == 0) ? H.timer : nullptr;
  dispatch_smooth<T, NV>(L, v, tr, s, 0, timer);
  dispatch_transfer<T, NV>(L, v, cv.lv[l + 1], s, true);
  vcycle_rec<T, NV>(H, cv, l + 1, tr, s);
  dispatch_transfer<T, NV>(L, v, cv.lv[l + 1], s, false);
  dispatch_smooth<T, NV>(L, v, tr, s, 1, nullptr);
}

template <typename T>
std::vector<CycleVecs<T>>& vec_sets(Hierarchy& H);
template <>
std::vector<CycleVecs<double>>& vec_sets<double>(Hierarchy& H) {
  return H.v64;
}
template <>
std::vector<CycleVecs<float>>& vec_sets<float>(Hierarchy& H) {
  return H.v32;
}

}  // namespace

template <typename T>
CycleVecs<T>& cycle_vecs(Hierarchy& H, int nv) {
  auto& sets = vec_sets<T>(H);
  for (auto& c : sets)
    if (c.nv == nv) return c;
  sets.emplace_back();
  CycleVecs<T>& c = sets.back();
  c.nv = nv;
  c.lv.resize(H.L.size());
  for (size_t l = 0; l < H.L.size(); ++l) {
    const int64_t n = H.L[l].n_nodes * H.L[l].bs * (int64_t)nv;
    LevelVecs<T>& v = c.lv[l];
    v.b.alloc(n);
    v.xo.alloc(n);
    if (!H.L[l].coarsest) {
      v.x.alloc(n);
      v.d.alloc(n);
      v.r.alloc(n);
      v.res.alloc(n);
    }
  }
  return c;
}
template CycleVecs<double>& cycle_vecs<double>(Hierarchy&, int);
template CycleVecs<float>& cycle_vecs<float>(Hierarchy&, int);

template <typename T, int NV>
void vcycle(Hierarchy& H, bool transpose, hipStream_t s) {
  CycleVecs<T>& cv = cycle_vecs<T>(H, NV);
  vcycle_rec<T, NV>(H, cv, 0, transpose, s);
}
template void vcycle<double, 1>(Hierarchy&, bool, hipStream_t);
template void vcycle<double, 2>(Hierarchy&, bool, hipStream_t);
template void vcycle<float, 1>(Hierarchy&, bool, hipStream_t);
template void vcycle<float, 2>(Hierarchy&, bool, hipStream_t);

void sell_mv(const Sell<double>& A, const double* x, double* y, hipStream_t s) {
  if (A.br == 3 && A.bc == 3)
    launch_sell<double, 3, 3, 1>(A, LoadX<double, 1>{x},
                                 EpiStore<double, 3, 1>{y}, s);
  else if (A.br == 6 && A.bc == 6)
    launch_sell<double, 6, 6, 1>(A, LoadX<double, 1>{x},
                                 EpiStore<double, 6, 1>{y}, s);
  else
    throw Error(FPC_ERR_ARG, "sell_mv: unsupported block shape");
}

void sell_mv_dinv(const Sell<double>& A, const double* dinv, const double* x,
                  double* y, hipStream_t s) {
  if (A.br == 3 && A.bc == 3)
    launch_sell<double, 3, 3, 1>(A, LoadX<double, 1>{x},
                                 EpiDinv<double, 3>{dinv, y}, s);
  else if (A.br == 6 && A.bc == 6)
    launch_sell<double, 6, 6, 1>(A, LoadX<double, 1>{x},
                                 EpiDinv<double, 6>{dinv, y}, s);
  else
    throw Error(FPC_ERR_ARG, "sell_mv_dinv: unsupported block shape");
}

void face_apply(const double* hinv, const double* in, double* out,
                int64_t n_p, int trans, hipStream_t s) {
  if (n_p == 0) return;
  k_face_apply<<<grid_for(n_p, 256), 256, 0, s>>>(hinv, in, out, n_p, trans);
  FPC_LAUNCH_CHECK();
}

template <typename T>
void to_level(T* out, int nv, int colv, int64_t n, const double* base,
              const Csr* m1, const double* x1, double a1, const Csr* m2,
              const double* x2, double a2, hipStream_t s) {
  if (n == 0) return;
  k_to_level<T><<<grid_for(n, 256), 256, 0, s>>>(
      out, nv, colv, base, m1 ? m1->rowptr.p : nullptr,
      m1 ? m1->col.p : nullptr, m1 ? m1->val.p : nullptr, x1, a1,
      m2 ? m2->rowptr.p : nullptr, m2 ? m2->col.p : nullptr,
      m2 ? m2->val.p : nullptr, x2, a2, n);
  FPC_LAUNCH_CHECK();
}
template void to_level<double>(double*, int, int, int64_t, const double*,
                               const Csr*, const double*, double, const Csr*,
                               const double*, double, hipStream_t);
template void to_level<float>(float*, int, int, int64_t, const double*,
                              const Csr*, const double*, double, const Csr*,
                              const double*, double, hipStream_t);

template <typename T>
void from_level(const T* xo, int nv, int64_t n, double* vu, int diff,
                hipStream_t s) {
  if (n == 0) return;
  k_from_level<T><<<grid_for(n, 256), 256, 0, s>>>(xo, nv, n, vu, diff);
  FPC_LAUNCH_CHECK();
}
template void from_level<double>(const double*, int, int64_t, double*, int,
                                 hipStream_t);
template void from_level<float>(const float*, int, int64_t, double*, int,
                                hipStream_t);

void tface(const Csr& C, const double* vu, const double* t_t,
           const double* hinv, double* v_t, int64_t n_p, int trans,
           hipStream_t s) {
  if (n_p == 0) return;
  k_tface<<<grid_for(n_p, 128), 128, 0, s>>>(C.rowptr.p, C.col.p, C.val.p, vu,
                                             t_t, hinv, v_t, n_p, trans);
  FPC_LAUNCH_CHECK();
}

void psolve_apply(const PSolve& ps, const double* in, double* out,
                  int64_t n_p, int trans, hipStream_t s) {
  if (n_p == 0) return;
  k_psolve<<<(unsigned)((n_p + 3) / 4), 256, 0, s>>>(
      ps.dense.p, ps.dense_off.p, ps.comp_off.p, ps.comp_pad_d.p,
      ps.comp_of_row.p, ps.members.p, in, out, n_p, trans);
  FPC_LAUNCH_CHECK();
}

}  // namespace fpc
