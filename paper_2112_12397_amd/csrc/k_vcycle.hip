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
  const int32_t* __restrict__ perm;  // null: position = row
};

template <typename T>
SellView<T> view(const Sell<T>& a) {
  return SellView<T>{a.nrows, a.nslices, a.slice_ptr.p, a.row_len.p,
                     a.col.p, a.val.p, a.perm.n ? a.perm.p : nullptr};
}

// The row stored at position `pos` of a sliced-ELL layout.
template <typename T>
__device__ __forceinline__ int64_t sell_row(const SellView<T>& A,
                                            int64_t pos) {
  return A.perm ? (int64_t)A.perm[pos] : pos;
}

// ---------------------------------------------------------------- loaders
template <typename T, int NV>
struct LoadX {
  const T* __restrict__ x;
  __device__ T operator()(int64_t dof, int v) const { return x[dof * NV + v]; }
};


// ---------------------------------------------------------------- epilogues
// Every epilogue works element-wise on (dof, column): element (dof, v) of an
// NV-column vector sits at k = dof * NV + v.  `load` fetches the element's
// inputs into registers, `eval` combines them with the product value `a`
// into NOUT outputs and `put(o, k, value)` writes output o.  Callers issue
// all loads of a row before any store, and write the outputs array by array
// in increasing k: the compiler may not move a store past a store through
// another pointer, so interleaved outputs would be written one element per
// instruction, while one array's consecutive elements merge into one wide
// store.
template <typename T, int NV>
struct EpiStore {
  static constexpr int NIN = 1, NOUT = 1;
  T* __restrict__ y;
  __device__ void load(int64_t, int64_t, T*) const {}
  __device__ void eval(int64_t, T a, const T*, T* out) const { out[0] = a; }
  __device__ void put(int, int64_t k, T val) const { y[k] = val; }
};

template <typename T, int NV>
struct EpiAdd {
  static constexpr int NIN = 1, NOUT = 1;
  T* __restrict__ y;
  __device__ void load(int64_t, int64_t k, T* in) const { in[0] = y[k]; }
  __device__ void eval(int64_t, T a, const T* in, T* out) const {
    out[0] = in[0] + a;
  }
  __device__ void put(int, int64_t k, T val) const { y[k] = val; }
};

// restriction onto a smoothed level: b = R res and the first Chebyshev
// direction d0 = D^{-1} b / theta of that level
template <typename T, int NV>
struct EpiRestrict {
  static constexpr int NIN = 1, NOUT = 2;
  T* __restrict__ b;
  T* __restrict__ d0;
  const T* __restrict__ dinv;
  T inv_theta;
  __device__ void load(int64_t dof, int64_t, T* in) const { in[0] = dinv[dof]; }
  __device__ void eval(int64_t, T a, const T* in, T* out) const {
    out[0] = a;
    out[1] = in[0] * a * inv_theta;
  }
  __device__ void put(int o, int64_t k, T val) const {
    if (o == 0) b[k] = val;
    else d0[k] = val;
  }
};

// y = D^{-1} (A x), one column
template <typename T, int NV>
struct EpiDinv {
  static constexpr int NIN = 1, NOUT = 1;
  const T* __restrict__ dinv;
  T* __restrict__ y;
  __device__ void load(int64_t dof, int64_t, T* in) const { in[0] = dinv[dof]; }
  __device__ void eval(int64_t, T a, const T* in, T* out) const {
    out[0] = in[0] * a;
  }
  __device__ void put(int, int64_t k, T val) const { y[k] = val; }
};

// Pre-smoothing from x = 0, two Chebyshev steps fused around q = A d0 (d0
// was written with b by the restriction, or by k_first_dir on level 0):
//   R1 = b - q, r1 = D^-1 R1, d1 = c1 d0 + c2 r1, x = d0 + d1.
template <typename T, int NV>
struct EpiPre1 {
  static constexpr int NIN = 2, NOUT = 3;
  const T* __restrict__ b;
  const T* __restrict__ dinv;
  T* __restrict__ x;
  T* __restrict__ d;
  T* __restrict__ R;
  T inv_theta, c1, c2;
  __device__ void load(int64_t dof, int64_t k, T* in) const {
    in[0] = b[k];
    in[1] = dinv[dof];
  }
  __device__ void eval(int64_t, T a, const T* in, T* out) const {
    const T bi = in[0], di = in[1];
    const T d0 = di * bi * inv_theta;
    const T R1 = bi - a;
    const T r1 = di * R1;
    const T d1 = c1 * d0 + c2 * r1;
    out[0] = d0 + d1;
    out[1] = d1;
    out[2] = R1;
  }
  __device__ void put(int o, int64_t k, T val) const {
    if (o == 0) x[k] = val;
    else if (o == 1) d[k] = val;
    else R[k] = val;
  }
};

// residual after pre-smoothing: res = R1 - A d1 = b - A x
template <typename T, int NV>
struct EpiRes {
  static constexpr int NIN = 1, NOUT = 1;
  const T* __restrict__ R;
  T* __restrict__ res;
  __device__ void load(int64_t, int64_t k, T* in) const { in[0] = R[k]; }
  __device__ void eval(int64_t, T a, const T* in, T* out) const {
    out[0] = in[0] - a;
  }
  __device__ void put(int, int64_t k, T val) const { res[k] = val; }
};

// post-smoothing step 1 around q = A x: r0 = D^-1 (b - q) and d0 = r0 /
// theta; only d0 is stored (r0 = theta d0 is formed again in step 2, and
// step 2 adds d0 to x itself)
template <typename T, int NV>
struct EpiPost1 {
  static constexpr int NIN = 2, NOUT = 1;
  const T* __restrict__ b;
  const T* __restrict__ dinv;
  T* __restrict__ d;
  T inv_theta;
  __device__ void load(int64_t dof, int64_t k, T* in) const {
    in[0] = b[k];
    in[1] = dinv[dof];
  }
  __device__ void eval(int64_t, T a, const T* in, T* out) const {
    out[0] = in[1] * (in[0] - a) * inv_theta;
  }
  __device__ void put(int, int64_t k, T val) const { d[k] = val; }
};

// post-smoothing step 2 around q = A d0: r1 = theta d0 - D^-1 q,
// d1 = c1 d0 + c2 r1, xo = (x + d0) + d1
template <typename T, int NV>
struct EpiPost2 {
  static constexpr int NIN = 3, NOUT = 1;
  const T* __restrict__ dinv;
  const T* __restrict__ din;
  const T* __restrict__ x;
  T* __restrict__ xo;
  T theta, c1, c2;
  __device__ void load(int64_t dof, int64_t k, T* in) const {
    in[0] = dinv[dof];
    in[1] = din[k];
    in[2] = x[k];
  }
  __device__ void eval(int64_t, T a, const T* in, T* out) const {
    const T d0 = in[1];
    const T r1 = theta * d0 - in[0] * a;
    out[0] = (in[2] + d0) + (c1 * d0 + c2 * r1);
  }
  __device__ void put(int, int64_t k, T val) const { xo[k] = val; }
};

// EpiPost2 on the finest level with the cycle's result written once, in
// FP64, to the caller's vector (rounded to T first, as a separate
// conversion of xo would do)
template <typename T, int NV>
struct EpiPost2Out {
  static constexpr int NIN = 3, NOUT = 1;
  const T* __restrict__ dinv;
  const T* __restrict__ din;
  const T* __restrict__ x;
  double* __restrict__ out;
  T theta, c1, c2;
  __device__ void load(int64_t dof, int64_t k, T* in) const {
    in[0] = dinv[dof];
    in[1] = din[k];
    in[2] = x[k];
  }
  __device__ void eval(int64_t, T a, const T* in, T* o) const {
    const T d0 = in[1];
    const T r1 = theta * d0 - in[0] * a;
    o[0] = (in[2] + d0) + (c1 * d0 + c2 * r1);
  }
  __device__ void put(int, int64_t k, T val) const { out[k] = (double)val; }
};

// The loads and the stores of one block row (all NV columns) as two steps,
// so that a kernel can issue the loads before its product and keep the
// inputs in registers.
template <typename T, int BR, int NV, class Epi>
__device__ inline void epi_load_row(const Epi& e, int64_t row,
                                    T (&in)[NV][BR][Epi::NIN]) {
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int i = 0; i < BR; ++i) {
      const int64_t dof = row * BR + i;
      e.load(dof, dof * NV + v, in[v][i]);
    }
}
template <typename T, int BR, int NV, class Epi>
__device__ inline void epi_store_row(const Epi& e, int64_t row,
                                     const T (&acc)[NV][BR],
                                     const T (&in)[NV][BR][Epi::NIN]) {
  T out[NV][BR][Epi::NOUT];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int i = 0; i < BR; ++i)
      e.eval(row * BR + i, acc[v][i], in[v][i], out[v][i]);
#pragma unroll
  for (int o = 0; o < Epi::NOUT; ++o)
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int v = 0; v < NV; ++v)
        e.put(o, (row * BR + i) * NV + v, out[v][i][o]);
}

// Columns v0 .. v0 + CPL - 1 of one block row.
template <typename T, int BR, int NV, int CPL, class Epi>
__device__ inline void epi_cols(const Epi& e, int64_t row, int v0,
                                const T (&acc)[CPL][BR]) {
  T in[CPL][BR][Epi::NIN];
  T out[CPL][BR][Epi::NOUT];
#pragma unroll
  for (int i = 0; i < BR; ++i)
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int64_t dof = row * BR + i;
      e.load(dof, dof * NV + v0 + u, in[u][i]);
    }
#pragma unroll
  for (int i = 0; i < BR; ++i)
#pragma unroll
    for (int u = 0; u < CPL; ++u)
      e.eval(row * BR + i, acc[u][i], in[u][i], out[u][i]);
#pragma unroll
  for (int o = 0; o < Epi::NOUT; ++o)
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int u = 0; u < CPL; ++u)
        e.put(o, (row * BR + i) * NV + v0 + u, out[u][i][o]);
}

// One element (component i, column v) of one block row.
template <typename T, int BR, int NV, class Epi>
__device__ inline void epi_one(const Epi& e, int64_t row, int i, int v, T a) {
  T in[Epi::NIN];
  T out[Epi::NOUT];
  const int64_t dof = row * BR + i;
  e.load(dof, dof * NV + v, in);
  e.eval(dof, a, in, out);
#pragma unroll
  for (int o = 0; o < Epi::NOUT; ++o) e.put(o, dof * NV + v, out[o]);
}

// ---------------------------------------------------------------- SpMV
// Streamed operands (matrix values and indices read once per product, larger
// than the last-level cache at the sizes that matter) are loaded with the
// nontemporal hint, so they do not evict the gathered vector.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}

// 3x3 sliced-ELL slots carry a class in bits 30-31 of the column index:
// 0 = nine values, 1 + i0 = five values (row and column i0 zero off the
// diagonal; planes m[i0][i0], m[i1][i1], m[i1][i2], m[i2][i1], m[i2][i2]).
// Only full slots read value planes 5-8.
__device__ __forceinline__ int slot_col(int32_t raw) { return raw & 0x3fffffff; }
__device__ __forceinline__ int slot_class(int32_t raw) {
  return (int)((uint32_t)raw >> 30);
}

template <typename T>
__device__ __forceinline__ void load33(const T* __restrict__ vb, int cls,
                                       T* m) {
  T p[9];
#pragma unroll
  for (int q = 0; q < 5; ++q) p[q] = ld_stream(vb + q * kSliceH);
  if (cls == 0) {
#pragma unroll
    for (int q = 5; q < 9; ++q) p[q] = ld_stream(vb + q * kSliceH);
  } else {
#pragma unroll
    for (int q = 5; q < 9; ++q) p[q] = T(0);
  }
  const bool f = cls == 0;
  const T z = T(0);
  m[0] = (f || cls == 1) ? p[0] : p[1];
  m[1] = f ? p[1] : (cls == 3 ? p[2] : z);
  m[2] = f ? p[2] : (cls == 2 ? p[2] : z);
  m[3] = f ? p[3] : (cls == 3 ? p[3] : z);
  m[4] = f ? p[4] : (cls == 1 ? p[1] : (cls == 2 ? p[0] : p[4]));
  m[5] = f ? p[5] : (cls == 1 ? p[2] : z);
  m[6] = f ? p[6] : (cls == 2 ? p[3] : z);
  m[7] = f ? p[7] : (cls == 1 ? p[3] : z);
  m[8] = f ? p[8] : (cls == 3 ? p[0] : p[4]);
}

constexpr int kSliceSplit = 4;

// Few columns (NV <= 2): kSliceSplit wavefronts per 64-row slice, one thread
// per block row carrying all NV columns, so each matrix block is read by one
// lane only.  Wavefront h of a slice takes slots h, h + kSliceSplit, ...
// (full and packed slots spread evenly) and hands its partial sums to
// wavefront 0 through LDS, which adds them in order and runs the epilogue; a
// whole slice per wavefront leaves too few wavefronts in flight to cover the
// memory latency.  Every lane runs to the slice's longest row: padding slots
// hold zero values and a column of their own row, so they need no guard.
// Slots are taken U at a time: the column indices of the next batch are
// fetched one batch ahead, then the x values and all block values of the
// batch are in flight together.
template <typename T, int BR, int BC, int NV, class Load, class Epi>
__global__ __launch_bounds__(256) void k_sell_rows(SellView<T> A, Load ld,
                                                   Epi epi) {
  constexpr int U = BR * BC <= 9 ? 3 : (BR * BC <= 18 ? 2 : 1);
  constexpr bool kPacked33 = BR == 3 && BC == 3;
  constexpr int SP = kSliceSplit;  // wavefronts per slice
  __shared__ T red[4 / SP][SP - 1][64][NV * BR];
  const int wave = threadIdx.x >> 6;
  const int half = wave % SP, pair = wave / SP;
  const int slice = __builtin_amdgcn_readfirstlane(
      (int)(xcd_block(blockIdx.x, gridDim.x) * (4 / SP) + pair));
  const bool valid = slice < A.nslices;
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)slice * kSliceH + lane;
  T acc[NV][BR];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int i = 0; i < BR; ++i) acc[v][i] = T(0);
  // the epilogue's inputs do not depend on the product: wavefront 0 fetches
  // them first, so they arrive while the slice streams in
  const bool epi_lane = half == 0 && valid && row < A.nrows;
  const int64_t orow = epi_lane ? sell_row(A, row) : 0;
  T pre[NV][BR][Epi::NIN];
  if (epi_lane) epi_load_row<T, BR, NV>(epi, orow, pre);
  if (valid) {
    const int64_t base = A.slice_ptr[slice];
    const int maxlen = (int)((A.slice_ptr[slice + 1] - base) / kSliceH);
    const int32_t* __restrict__ cp = A.col + base + lane;
    const T* __restrict__ vp = A.val + base * (BR * BC) + lane;
    int cn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = half + SP * u;
      cn[u] = k < maxlen ? ld_stream(cp + (int64_t)k * kSliceH) : 0;
    }
    for (int k0 = half; k0 < maxlen; k0 += SP * U) {
      int cc[U];
#pragma unroll
      for (int u = 0; u < U; ++u) cc[u] = cn[u];
      T xv[U][BC][NV];
      T a[U][BR * BC];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + SP * u;
        if (k < maxlen) {
          const int64_t col = kPacked33 ? slot_col(cc[u]) : cc[u];
#pragma unroll
          for (int j = 0; j < BC; ++j)
#pragma unroll
            for (int v = 0; v < NV; ++v) xv[u][j][v] = ld(col * BC + j, v);
          const T* __restrict__ vb = vp + (int64_t)k * kSliceH * (BR * BC);
          if constexpr (kPacked33) {
            load33(vb, slot_class(cc[u]), a[u]);
          } else {
#pragma unroll
            for (int q = 0; q < BR * BC; ++q) a[u][q] = ld_stream(vb + q * kSliceH);
          }
        } else {
#pragma unroll
          for (int j = 0; j < BC; ++j)
#pragma unroll
            for (int v = 0; v < NV; ++v) xv[u][j][v] = T(0);
#pragma unroll
          for (int q = 0; q < BR * BC; ++q) a[u][q] = T(0);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int kn = k0 + SP * U + SP * u;
        cn[u] = kn < maxlen ? ld_stream(cp + (int64_t)kn * kSliceH) : 0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int i = 0; i < BR; ++i)
#pragma unroll
          for (int j = 0; j < BC; ++j)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v][i] += a[u][i * BC + j] * xv[u][j][v];
    }
  }
  if (half > 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int i = 0; i < BR; ++i) red[pair][half - 1][lane][v * BR + i] = acc[v][i];
  }
  __syncthreads();
  if (!epi_lane) return;
#pragma unroll
  for (int h = 0; h < SP - 1; ++h)
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int i = 0; i < BR; ++i) acc[v][i] += red[pair][h][lane][v * BR + i];
  epi_store_row<T, BR, NV>(epi, orow, acc, pre);
}

// Many columns (interleaved right-hand sides): one thread per (block row,
// CPL consecutive columns); a wavefront covers 64 CPL / NV consecutive block
// rows of one slice, so the columns of one x row are read as one contiguous
// segment and every matrix block is broadcast to the NV / CPL lanes of its
// row.  For 3x3 blocks from 16 columns on a lane takes 16 bytes of columns
// (four FP32 or two FP64), fetched as one load per x row, which also cuts
// the matrix loads per column (larger blocks keep one column per lane:
// their registers would not hold more).
template <typename T, int BR, int BC, int NV>
constexpr int sell_cols_cpl() {
  return (NV >= 16 && BR * BC <= 9) ? (int)(16 / sizeof(T)) : 1;
}

// CPL consecutive elements of one x row as a single (16-byte) load
template <typename T, int CPL>
struct alignas(sizeof(T) * CPL) XPack {
  T v[CPL];
};

template <typename T, int BR, int BC, int NV, class Load, class Epi>
__global__ __launch_bounds__(256) void k_sell_cols(SellView<T> A, Load ld,
                                                   Epi epi) {
  constexpr int CPL = sell_cols_cpl<T, BR, BC, NV>();
  constexpr int LPR = NV / CPL;  // lanes per block row
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t gw = blk * 4 + wave;
  const int64_t slice = gw / LPR;
  if (slice >= A.nslices) return;
  const int sub = (int)(gw % LPR);
  const int rloc = sub * (64 / LPR) + lane / LPR;
  const int v0 = (lane % LPR) * CPL;
  const int64_t row = slice * kSliceH + rloc;
  if (row >= A.nrows) return;
  const int len = A.row_len[row];
  const int64_t base = A.slice_ptr[slice];
  const int32_t* __restrict__ cp = A.col + base + rloc;
  const T* __restrict__ vp = A.val + base * (BR * BC) + rloc;
  T acc[CPL][BR];
#pragma unroll
  for (int u = 0; u < CPL; ++u)
#pragma unroll
    for (int i = 0; i < BR; ++i) acc[u][i] = T(0);
#pragma unroll 2
  for (int k = 0; k < len; ++k) {
    const int32_t raw = cp[(int64_t)k * kSliceH];
    const int64_t c = (BR == 3 && BC == 3) ? slot_col(raw) : raw;
    const T* __restrict__ vb = vp + (int64_t)k * kSliceH * (BR * BC);
    T xv[BC][CPL];
    if constexpr (CPL > 1) {
#pragma unroll
      for (int j = 0; j < BC; ++j) {
        const XPack<T, CPL> q = *reinterpret_cast<const XPack<T, CPL>*>(
            ld.x + (c * BC + j) * NV + v0);
#pragma unroll
        for (int u = 0; u < CPL; ++u) xv[j][u] = q.v[u];
      }
    } else {
#pragma unroll
      for (int j = 0; j < BC; ++j) xv[j][0] = ld(c * BC + j, v0);
    }
    T m[BR * BC];
    if constexpr (BR == 3 && BC == 3) {
      load33(vb, slot_class(raw), m);
    } else {
#pragma unroll
      for (int q = 0; q < BR * BC; ++q) m[q] = vb[q * kSliceH];
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u)
#pragma unroll
      for (int i = 0; i < BR; ++i)
#pragma unroll
        for (int j = 0; j < BC; ++j) acc[u][i] += m[i * BC + j] * xv[j][u];
  }
  epi_cols<T, BR, NV, CPL>(epi, sell_row(A, row), v0, acc);
}

template <typename T, int BR, int BC, int NV, class Load, class Epi>
void launch_sell(const Sell<T>& A, Load ld, Epi epi, hipStream_t s) {
  if (A.nrows == 0) return;
  if constexpr (NV <= 2) {
    const unsigned grid =
        (unsigned)((A.nslices + 4 / kSliceSplit - 1) / (4 / kSliceSplit));
    k_sell_rows<T, BR, BC, NV, Load, Epi><<<grid, 256, 0, s>>>(view(A), ld, epi);
  } else {
    const int64_t waves = A.nslices * (NV / sell_cols_cpl<T, BR, BC, NV>());
    const unsigned grid = (unsigned)((waves + 3) / 4);
    k_sell_cols<T, BR, BC, NV, Load, Epi><<<grid, 256, 0, s>>>(view(A), ld, epi);
  }
  FPC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- row groups
template <typename T>
struct VrowView {
  int64_t nrows;
  const int64_t* __restrict__ chunk_ptr;
  const int32_t* __restrict__ row_len;
  const int32_t* __restrict__ col;
  const T* __restrict__ val;
};

template <typename T>
VrowView<T> vview(const Vrow<T>& a) {
  return VrowView<T>{a.nrows, a.chunk_ptr.p, a.row_len.p, a.col.p, a.val.p};
}

// G lanes per block row: lane sl takes blocks sl, sl+G, ... of the row
// (chunk-contiguous, component-major), then the G partial sums are combined
// with cross-lane shuffles inside the aligned lane group; with G = 256 (a
// workgroup per row, for the few long rows of coarse restrictions) the four
// wavefronts' sums then meet in LDS and are added in wavefront order.
template <typename T, int BR, int BC, int NV, int G, class Load, class Epi>
__global__ __launch_bounds__(256) void k_vrow(VrowView<T> A, Load ld, Epi epi) {
  static_assert(G <= 64 || G == 256, "row groups: up to 64 lanes, or 256");
  constexpr int GW = G > 64 ? 64 : G;  // lanes combined by shuffles
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t t = blk * 256 + threadIdx.x;
  const int64_t row = t / G;
  const int sl = (int)(t % G);
  if (row >= A.nrows) return;
  const int len = A.row_len[row];
  const int64_t c0 = A.chunk_ptr[row];
  T acc[NV][BR];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int i = 0; i < BR; ++i) acc[v][i] = T(0);
  for (int k0 = 0; k0 < len; k0 += G) {
    if (k0 + sl < len) {
      const int64_t grp = (c0 + k0 / G) * (int64_t)G;
      const int64_t c = A.col[grp + sl];
      const T* __restrict__ vb = A.val + grp * (BR * BC) + sl;
      T bv[BR * BC];
#pragma unroll
      for (int q = 0; q < BR * BC; ++q) bv[q] = vb[(int64_t)q * G];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        T xv[BC];
#pragma unroll
        for (int j = 0; j < BC; ++j) xv[j] = ld(c * BC + j, v);
#pragma unroll
        for (int i = 0; i < BR; ++i)
#pragma unroll
          for (int j = 0; j < BC; ++j) acc[v][i] += bv[i * BC + j] * xv[j];
      }
    }
  }
#pragma unroll
  for (int off = GW / 2; off > 0; off >>= 1)
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int i = 0; i < BR; ++i) acc[v][i] += __shfl_xor(acc[v][i], off, 64);
  if constexpr (G == 256) {
    __shared__ T red[4][BR * NV];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int i = 0; i < BR; ++i) red[w][i * NV + v] = acc[v][i];
    __syncthreads();
    if (threadIdx.x < BR * NV) {
      const int q = threadIdx.x;
      const T a = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
      epi_one<T, BR, NV>(epi, row, q / NV, q % NV, a);
    }
    return;
  }
  // after the butterfly every lane of the group holds all BR*NV sums; lane
  // sl writes elements sl, sl+G, ...
#pragma unroll
  for (int q0 = 0; q0 < BR * NV; q0 += G) {
    const int q = q0 + sl;
    if (q < BR * NV) {
      T a = T(0);
#pragma unroll
      for (int vv = 0; vv < NV; ++vv)
#pragma unroll
        for (int ii = 0; ii < BR; ++ii)
          if (ii * NV + vv == q) a = acc[vv][ii];
      epi_one<T, BR, NV>(epi, row, q / NV, q % NV, a);
    }
  }
}

// Many columns on the row-group layout (operators with long rows, such as
// the restrictions): one wavefront per block row; lane = g + G cg with G =
// kBatchRowGroup, the G lanes g split the row's blocks (chunks of G,
// component-major, so the G lanes of a column group read G consecutive
// words and the 8 column groups share them) and column group cg takes the
// NV / 8 consecutive columns from v0 = cg NV / 8 (16- or 32-byte x loads
// for 32 columns); the G partial sums are combined by shuffles and lane
// g = 0 of each group runs the epilogue.
template <typename T, int BR, int BC, int NV, int WPR, class Load, class Epi>
__global__ __launch_bounds__(256) void k_vrow_cols(VrowView<T> A, Load ld,
                                                   Epi epi) {
  constexpr int G = kBatchRowGroup;
  constexpr int CPL = NV / (64 / G);
  static_assert(CPL >= 1 && CPL * (64 / G) == NV, "one wavefront per row");
  // WPR wavefronts per row (rows of hundreds of blocks): wavefront h takes
  // chunks h, h + WPR, ...; their sums are added in order through LDS
  __shared__ T red[WPR > 1 ? 4 : 1][64 / G][CPL * BR];
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int wave = threadIdx.x >> 6;
  const int64_t row = blk * (4 / WPR) + wave / WPR;
  const int h = wave % WPR;
  const bool live = row < A.nrows;
  if (WPR == 1 && !live) return;
  const int lane = threadIdx.x & 63;
  const int g = lane % G, cg = lane / G;
  const int v0 = cg * CPL;
  T acc[CPL][BR];
#pragma unroll
  for (int u = 0; u < CPL; ++u)
#pragma unroll
    for (int i = 0; i < BR; ++i) acc[u][i] = T(0);
  if (live) {
    const int len = A.row_len[row];
    const int64_t c0 = A.chunk_ptr[row];
    for (int k0 = h * G; k0 < len; k0 += G * WPR) {
      if (k0 + g < len) {
        const int64_t grp = (c0 + k0 / G) * (int64_t)G;
        const int64_t c = A.col[grp + g];
        const T* __restrict__ vb = A.val + grp * (BR * BC) + g;
        T m[BR * BC];
#pragma unroll
        for (int q = 0; q < BR * BC; ++q) m[q] = vb[(int64_t)q * G];
        T xv[BC][CPL];
        if constexpr (CPL > 1) {
#pragma unroll
          for (int j = 0; j < BC; ++j) {
            const XPack<T, CPL> xp = *reinterpret_cast<const XPack<T, CPL>*>(
                ld.x + (c * BC + j) * NV + v0);
#pragma unroll
            for (int u = 0; u < CPL; ++u) xv[j][u] = xp.v[u];
          }
        } else {
#pragma unroll
          for (int j = 0; j < BC; ++j) xv[j][0] = ld(c * BC + j, v0);
        }
#pragma unroll
        for (int u = 0; u < CPL; ++u)
#pragma unroll
          for (int i = 0; i < BR; ++i)
#pragma unroll
            for (int j = 0; j < BC; ++j) acc[u][i] += m[i * BC + j] * xv[j][u];
      }
    }
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1)
#pragma unroll
    for (int u = 0; u < CPL; ++u)
#pragma unroll
      for (int i = 0; i < BR; ++i) acc[u][i] += __shfl_xor(acc[u][i], off, 64);
  if constexpr (WPR > 1) {
    if (g == 0)
#pragma unroll
      for (int u = 0; u < CPL; ++u)
#pragma unroll
        for (int i = 0; i < BR; ++i) red[wave][cg][u * BR + i] = acc[u][i];
    __syncthreads();
    if (h != 0 || !live) return;
#pragma unroll
    for (int u = 0; u < CPL; ++u)
#pragma unroll
      for (int i = 0; i < BR; ++i) {
        T t = red[wave][cg][u * BR + i];
#pragma unroll
        for (int q = 1; q < WPR; ++q) t += red[wave + q][cg][u * BR + i];
        acc[u][i] = t;
      }
  }
  if (g == 0) epi_cols<T, BR, NV, CPL>(epi, row, v0, acc);
}

template <typename T, int BR, int BC, int NV, class Load, class Epi>
void launch_vrow_cols(const Vrow<T>& A, int wpr, Load ld, Epi epi,
                      hipStream_t s) {
  if (A.nrows == 0) return;
  if (A.G != kBatchRowGroup)
    throw Error(FPC_ERR_ARG, "launch_vrow_cols: row-group width");
  if (wpr == 4) {
    const unsigned grid = (unsigned)A.nrows;
    k_vrow_cols<T, BR, BC, NV, 4, Load, Epi><<<grid, 256, 0, s>>>(vview(A), ld,
                                                                  epi);
  } else {
    const unsigned grid = (unsigned)((A.nrows + 3) / 4);
    k_vrow_cols<T, BR, BC, NV, 1, Load, Epi><<<grid, 256, 0, s>>>(vview(A), ld,
                                                                  epi);
  }
  FPC_LAUNCH_CHECK();
}

template <typename T, int BR, int BC, int NV, int G, class Load, class Epi>
void launch_vrow(const Vrow<T>& A, Load ld, Epi epi, hipStream_t s) {
  if (A.nrows == 0) return;
  const int64_t threads = A.nrows * G;
  const unsigned grid = (unsigned)((threads + 255) / 256);
  k_vrow<T, BR, BC, NV, G, Load, Epi><<<grid, 256, 0, s>>>(vview(A), ld, epi);
  FPC_LAUNCH_CHECK();
}

template <typename T, int BR, int BC, int NV, class Load, class Epi>
void launch_op(const Op<T>& op, Load ld, Epi epi, hipStream_t s) {
  if constexpr (NV > 2) {
    // many columns: sliced ELL (one thread per row and column group), or
    // one (fmt 1) or four (fmt 2) wavefronts per row on the row-group layout
    if (op.fmt == 0) return launch_sell<T, BR, BC, NV>(op.s, ld, epi, s);
    return launch_vrow_cols<T, BR, BC, NV>(op.v, op.fmt == 2 ? 4 : 1, ld, epi,
                                           s);
  } else {
  if (op.fmt == 0) return launch_sell<T, BR, BC, NV>(op.s, ld, epi, s);
  switch (op.v.G) {
    case 4: return launch_vrow<T, BR, BC, NV, 4>(op.v, ld, epi, s);
    case 16: return launch_vrow<T, BR, BC, NV, 16>(op.v, ld, epi, s);
    case 64: return launch_vrow<T, BR, BC, NV, 64>(op.v, ld, epi, s);
    case 256: return launch_vrow<T, BR, BC, NV, 256>(op.v, ld, epi, s);
  }
  throw Error(FPC_ERR_ARG, "launch_op: unsupported row-group width");
  }
}

// ---------------------------------------------------------------- coarsest
// x = Ainv b on the coarsest level (FP64 arithmetic), one workgroup per row
// (the level has at most a few thousand rows: a wavefront per row left too
// few loads in flight).  Thread t adds the elements k = t, t + 256, ... in
// order, fetched CU at a time; the four wavefronts' sums are added in order.
template <typename T, int NV>
__global__ __launch_bounds__(256) void k_coarse(const double* __restrict__ Ai,
                                                int64_t ld, int64_t n,
                                                const T* __restrict__ b,
                                                T* __restrict__ x) {
  constexpr int CU = NV >= 8 ? 1 : 8;
  __shared__ double red[4][NV];
  const int64_t row = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  const double* __restrict__ a = Ai + row * ld;
  for (int64_t k0 = t; k0 < n; k0 += 256 * CU) {
    double m[CU];
    T bv[CU][NV];
#pragma unroll
    for (int u = 0; u < CU; ++u) {
      const int64_t k = k0 + 256 * u;
      const bool in = k < n;
      m[u] = in ? a[k] : 0.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) bv[u][v] = in ? b[k * NV + v] : T(0);
    }
#pragma unroll
    for (int u = 0; u < CU; ++u)
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += m[u] * (double)bv[u][v];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double r = acc[v];
    for (int off = 32; off > 0; off >>= 1) r += __shfl_xor(r, off, 64);
    if (lane == 0) red[wave][v] = r;
  }
  __syncthreads();
  if (t < NV)
    x[row * NV + t] = (T)((red[0][t] + red[1][t]) + (red[2][t] + red[3][t]));
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
    const double s = csr_row_sum(c1, v1, x1, rp1[i], rp1[i + 1]);
    r += a1 * s;
  }
  if (rp2) {
    const double s = csr_row_sum(c2, v2, x2, rp2[i], rp2[i + 1]);
    r += a2 * s;
  }
  out[i * nv + colv] = (T)r;
}

template <typename T>
__global__ void k_base_copy(T* __restrict__ out, int nv, int colv,
                            const double* __restrict__ base, int64_t n,
                            T* __restrict__ d0, const T* __restrict__ dinv,
                            T inv_theta) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T b = (T)(base ? base[i] : 0.0);
  out[i * nv + colv] = b;
  // the first Chebyshev direction of the finest level (as k_first_dir)
  if (d0) d0[i] = dinv[i] * b * inv_theta;
}

// k_to_level on the rows of two lists only: threads [0, nr1) take the rows
// where m1 is nonempty, threads [nr1, nr1 + nr2) the listed rows of m2
// where m1 is empty; same arithmetic per row.
template <typename T>
__global__ void k_to_level_rows(T* __restrict__ out, int nv, int colv,
                                const double* __restrict__ base,
                                const int32_t* rows1, int64_t nr1,
                                const int32_t* rows2, int64_t nr2,
                                const int64_t* rp1, const int32_t* c1,
                                const double* v1, const double* x1, double a1,
                                const int64_t* rp2, const int32_t* c2,
                                const double* v2, const double* x2, double a2,
                                T* __restrict__ d0, const T* __restrict__ dinv,
                                T inv_theta) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nr1 + nr2) return;
  const bool second = t >= nr1;
  const int64_t i = second ? rows2[t - nr1] : rows1[t];
  if (second && rp1 && rp1[i] < rp1[i + 1]) return;
  double r = base ? base[i] : 0.0;
  if (rp1) {
    const double s = csr_row_sum(c1, v1, x1, rp1[i], rp1[i + 1]);
    r += a1 * s;
  }
  if (rp2) {
    const double s = csr_row_sum(c2, v2, x2, rp2[i], rp2[i + 1]);
    r += a2 * s;
  }
  const T b = (T)r;
  out[i * nv + colv] = b;
  if (d0) d0[i] = dinv[i] * b * inv_theta;
}

template <typename T>
__global__ void k_from_level(const T* __restrict__ xo, int nv, int64_t n,
                             double* __restrict__ vu, int diff) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  vu[i] = diff ? (double)xo[i * nv] - (double)xo[i * nv + 1] : (double)xo[i * nv];
}

// v_t = -t_t + H~^{-1} (C v_u) face by face (Alg 3.4 steps 9-10): thread
// (face K, row r) forms s_r = (C v_u)[3K + r]; the three s of a face meet in
// LDS and each thread writes its row of v_t.  A block holds 64 faces.
__global__ __launch_bounds__(192) void k_tface(const int64_t* __restrict__ rp,
                                               const int32_t* __restrict__ col,
                                               const double* __restrict__ val,
                                               const double* __restrict__ vu,
                                               const double* __restrict__ t_t,
                                               const double* __restrict__ hinv,
                                               double* __restrict__ v_t,
                                               int64_t n_p, int trans) {
  __shared__ double sh[192];
  const int64_t K = (int64_t)blockIdx.x * 64 + threadIdx.x / 3;
  const int r = threadIdx.x % 3;
  const bool act = K < n_p;
  double a = 0.0;
  if (act) {
    const int64_t row = 3 * K + r;
    a = csr_row_sum(col, val, vu, rp[row], rp[row + 1]);
  }
  sh[threadIdx.x] = a;
  __syncthreads();
  if (!act) return;
  const double* s3 = sh + (threadIdx.x - r);
  const double* h = hinv + K * 9;
  const double hv = trans ? h[0 * 3 + r] * s3[0] + h[1 * 3 + r] * s3[1] + h[2 * 3 + r] * s3[2]
                          : h[r * 3 + 0] * s3[0] + h[r * 3 + 1] * s3[1] + h[r * 3 + 2] * s3[2];
  v_t[3 * K + r] = -t_t[3 * K + r] + hv;
}

template <typename T, int NV>
__global__ void k_zero(T* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * NV) p[i] = T(0);
}

// ---------------------------------------------------------------- V-cycle
template <typename T>
const Op<T>& selA(const Level& L, bool tr, bool batch);
template <>
const Op<double>& selA<double>(const Level& L, bool tr, bool batch) {
  return batch ? L.bA : (tr ? L.oAT : L.oA);
}
template <>
const Op<float>& selA<float>(const Level& L, bool tr, bool batch) {
  return batch ? L.gA : (tr ? L.fAT : L.fA);
}
template <typename T>
const Op<T>& selP(const Level& L, bool batch);
template <>
const Op<double>& selP<double>(const Level& L, bool batch) {
  return batch ? L.bP : L.oP;
}
template <>
const Op<float>& selP<float>(const Level& L, bool batch) {
  return batch ? L.gP : L.fP;
}
template <typename T>
const Op<T>& selR(const Level& L, bool batch);
template <>
const Op<double>& selR<double>(const Level& L, bool batch) {
  return batch ? L.bR : L.oR;
}
template <>
const Op<float>& selR<float>(const Level& L, bool batch) {
  return batch ? L.gR : L.fR;
}
template <typename T>
const T* seldinv(const Level& L);
template <>
const double* seldinv<double>(const Level& L) { return L.dinv.p; }
template <>
const float* seldinv<float>(const Level& L) { return L.dinv32.p; }

template <typename T, int BS, int NV>
void smooth_level(const Level& L, LevelVecs<T>& v, bool tr, hipStream_t s,
                  int phase, KTimer* timer, double* out = nullptr) {
  const Op<T>& A = selA<T>(L, tr, NV > 2);
  const T* dinv = seldinv<T>(L);
  const T it = T(1.0 / L.theta), c1 = T(L.c1), c2 = T(L.c2);
  if (phase == 0) {
    launch_op<T, BS, BS, NV>(A, LoadX<T, NV>{v.d0.p},
                               EpiPre1<T, NV>{v.b.p, dinv, v.x.p, v.d.p,
                                                  v.r.p, it, c1, c2},
                               s);
    if (timer) timer->begin(s);
    launch_op<T, BS, BS, NV>(A, LoadX<T, NV>{v.d.p},
                               EpiRes<T, NV>{v.r.p, v.res.p}, s);
    if (timer) timer->end(s);
  } else {
    launch_op<T, BS, BS, NV>(A, LoadX<T, NV>{v.x.p},
                               EpiPost1<T, NV>{v.b.p, dinv, v.d.p, it}, s);
    if (NV == 1 && out)
      launch_op<T, BS, BS, NV>(A, LoadX<T, NV>{v.d.p},
                                 EpiPost2Out<T, NV>{dinv, v.d.p, v.x.p, out,
                                                    T(L.theta), c1, c2},
                                 s);
    else
      launch_op<T, BS, BS, NV>(A, LoadX<T, NV>{v.d.p},
                                 EpiPost2<T, NV>{dinv, v.d.p, v.x.p, v.xo.p,
                                                     T(L.theta), c1, c2},
                                 s);
  }
}

template <typename T, int BS, int NB, int NV>
void restrict_level(const Level& L, const Level& Lc, LevelVecs<T>& v,
                    LevelVecs<T>& vc, hipStream_t s) {
  if (Lc.coarsest) {
    launch_op<T, NB, BS, NV>(selR<T>(L, NV > 2), LoadX<T, NV>{v.res.p},
                               EpiStore<T, NV>{vc.b.p}, s);
  } else {
    launch_op<T, NB, BS, NV>(
        selR<T>(L, NV > 2), LoadX<T, NV>{v.res.p},
        EpiRestrict<T, NV>{vc.b.p, vc.d0.p, seldinv<T>(Lc),
                               T(1.0 / Lc.theta)},
        s);
  }
}

template <typename T, int BS, int NB, int NV>
void prolong_level(const Level& L, LevelVecs<T>& v, LevelVecs<T>& vc,
                   hipStream_t s) {
  launch_op<T, BS, NB, NV>(selP<T>(L, NV > 2), LoadX<T, NV>{vc.xo.p},
                             EpiAdd<T, NV>{v.x.p}, s);
}

template <typename T, int NV>
void dispatch_smooth(const Level& L, LevelVecs<T>& v, bool tr, hipStream_t s,
                     int phase, KTimer* timer, double* out = nullptr) {
  if (L.bs == 3) smooth_level<T, 3, NV>(L, v, tr, s, phase, timer, out);
  else smooth_level<T, 6, NV>(L, v, tr, s, phase, timer, out);
}

template <typename T, int NV>
void dispatch_transfer(const Level& L, const Level& Lc, LevelVecs<T>& v,
                       LevelVecs<T>& vc, hipStream_t s, bool restr) {
  if (L.bs == 3 && L.nb == 6) {
    if (restr) restrict_level<T, 3, 6, NV>(L, Lc, v, vc, s);
    else prolong_level<T, 3, 6, NV>(L, v, vc, s);
  } else if (L.bs == 3 && L.nb == 3) {
    if (restr) restrict_level<T, 3, 3, NV>(L, Lc, v, vc, s);
    else prolong_level<T, 3, 3, NV>(L, v, vc, s);
  } else {
    if (restr) restrict_level<T, 6, 6, NV>(L, Lc, v, vc, s);
    else prolong_level<T, 6, 6, NV>(L, v, vc, s);
  }
}

// d0 = D^{-1} b / theta on the finest level, whose b the caller wrote
template <typename T, int NV>
__global__ void k_first_dir(const T* __restrict__ b, const T* __restrict__ dinv,
                            T inv_theta, T* __restrict__ d0, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * NV) d0[i] = dinv[i / NV] * b[i] * inv_theta;
}

// Options of a single-column cycle: the finest level's first Chebyshev
// direction already formed (vcycle_input), and the result written in FP64
// to out by the last smoothing product instead of the finest level's xo.
struct CycleEnds {
  bool d0_ready = false;
  double* out = nullptr;
};

template <typename T, int NV>
void vcycle_rec(Hierarchy& H, CycleVecs<T>& cv, size_t l, bool tr,
                hipStream_t s, const CycleEnds& ends = CycleEnds{}) {
  const Level& L = H.L[l];
  LevelVecs<T>& v = cv.lv[l];
  if (L.coarsest) {
    const double* Ai = tr ? H.AinvT.p : H.Ainv.p;
    if (H.nc > 0)
      k_coarse<T, NV><<<(unsigned)H.nc, 256, 0, s>>>(Ai, H.ncpad, H.nc,
                                                     v.b.p, v.xo.p);
    FPC_LAUNCH_CHECK();
    return;
  }
  KTimer* timer = (l == 0) ? H.timer : nullptr;
  if (l == 0 && !ends.d0_ready) {
    const int64_t n = L.n_nodes * L.bs;
    k_first_dir<T, NV><<<grid_for(n * NV, 256), 256, 0, s>>>(
        v.b.p, seldinv<T>(L), T(1.0 / L.theta), v.d0.p, n);
    FPC_LAUNCH_CHECK();
  }
  dispatch_smooth<T, NV>(L, v, tr, s, 0, timer);
  const Level& Lc = H.L[l + 1];
  dispatch_transfer<T, NV>(L, Lc, v, cv.lv[l + 1], s, true);
  vcycle_rec<T, NV>(H, cv, l + 1, tr, s);
  dispatch_transfer<T, NV>(L, Lc, v, cv.lv[l + 1], s, false);
  dispatch_smooth<T, NV>(L, v, tr, s, 1, nullptr, l == 0 ? ends.out : nullptr);
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

// ---------------------------------------------------------------- tuner
template <typename T, int BR, int BC, int NV>
double time_op(const Op<T>& op, const T* x, T* y, hipStream_t s, int reps) {
  launch_op<T, BR, BC, NV>(op, LoadX<T, NV>{x}, EpiStore<T, NV>{y}, s);
  hipEvent_t e0, e1;
  FPC_HIP(hipEventCreate(&e0));
  FPC_HIP(hipEventCreate(&e1));
  FPC_HIP(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r)
    launch_op<T, BR, BC, NV>(op, LoadX<T, NV>{x}, EpiStore<T, NV>{y}, s);
  FPC_HIP(hipEventRecord(e1, s));
  FPC_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  FPC_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

template <typename T, int NV>
double time_any(const Op<T>& op, int br, int bc, const T* x, T* y,
                hipStream_t s, int reps) {
  if (br == 3 && bc == 3) return time_op<T, 3, 3, NV>(op, x, y, s, reps);
  if (br == 3 && bc == 6) return time_op<T, 3, 6, NV>(op, x, y, s, reps);
  if (br == 6 && bc == 3) return time_op<T, 6, 3, NV>(op, x, y, s, reps);
  if (br == 6 && bc == 6) return time_op<T, 6, 6, NV>(op, x, y, s, reps);
  throw Error(FPC_ERR_ARG, "tuner: unsupported block shape");
}

}  // namespace

// Pick the apply layout of one operator: sliced ELL (one thread per block
// row) or row groups of 4, 16 or 64 lanes, by timing `reps` products with
// `nv` columns on the device; only the winner is kept.
template <typename T>
void tune_op(const Bsr& M, int nv, Op<T>& out, hipStream_t s, int* choice,
             double* best_us, Sell<T>* sell) {
  DevBuf<T> x(std::max<int64_t>(M.nbc * M.bc * nv, 1));
  DevBuf<T> y(std::max<int64_t>(M.nbr * M.br * nv, 1));
  FPC_HIP(hipMemsetAsync(x.p, 0, x.bytes(), s));
  const int reps = 3;
  auto timeit = [&](const Op<T>& op) {
    return nv == 2 ? time_any<T, 2>(op, M.br, M.bc, x.p, y.p, s, reps)
                   : time_any<T, 1>(op, M.br, M.bc, x.p, y.p, s, reps);
  };
  // candidates that cannot win are skipped: sliced ELL for very long rows,
  // row groups wider than the average row
  const double avg = M.nbr ? (double)M.nnzb / (double)M.nbr : 0.0;
  Op<T> best;
  double tbest = 1e300;
  int cbest = 0;
  if (avg <= 64.0) {
    best.fmt = 0;
    if (sell && sell->nrows == M.nbr) best.s = std::move(*sell);
    else bsr_to_sell(M, best.s, s);
    tbest = timeit(best);
    cbest = 1;
  }
  for (int G : {4, 16, 64}) {
    // groups wider than the average row leave lanes idle
    if (cbest != 0 && G > avg) continue;
    Op<T> cand;
    cand.fmt = 1;
    bsr_to_vrow(M, G, cand.v, s);
    const double t = timeit(cand);
    if (t < tbest) {
      tbest = t;
      best = std::move(cand);
      cbest = G;
    } else if (cbest == 1 && t > 1.25 * tbest) {
      break;  // rows short enough for sliced ELL: wider groups only lose more
    }
  }
  out = std::move(best);
  if (choice) *choice = cbest;
  if (best_us) *best_us = 1e3 * tbest;
  FPC_HIP(hipStreamSynchronize(s));
}
int rule_layout(const Bsr& M, bool any_rows) {
  const double avg = M.nbr ? (double)M.nnzb / (double)M.nbr : 0.0;
  if (avg > 32.0)
    return avg < 64.0 ? 16 : (avg >= 256.0 && M.nbr < 4096) ? 256 : 64;
  if (any_rows || M.nbr >= 65536) return 1;
  return avg >= 16.0 ? 16 : 4;
}
template <typename T>
void build_op(const Bsr& M, int choice, Op<T>& out, hipStream_t s,
              Sell<T>* sell) {
  out = Op<T>();
  if (choice == 1) {
    out.fmt = 0;
    if (sell && sell->nrows == M.nbr) out.s = std::move(*sell);
    else bsr_to_sell(M, out.s, s);
  } else if (choice == 4 || choice == 16 || choice == 64 || choice == 256) {
    out.fmt = 1;
    bsr_to_vrow(M, choice, out.v, s);
  } else {
    throw Error(FPC_ERR_ARG, "build_op: unknown layout");
  }
}
template void build_op<double>(const Bsr&, int, Op<double>&, hipStream_t,
                               Sell<double>*);
template void build_op<float>(const Bsr&, int, Op<float>&, hipStream_t,
                              Sell<float>*);

template void tune_op<double>(const Bsr&, int, Op<double>&, hipStream_t, int*,
                              double*, Sell<double>*);
template void tune_op<float>(const Bsr&, int, Op<float>&, hipStream_t, int*,
                             double*, Sell<float>*);

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
      v.d0.alloc(n);
    }
  }
  return c;
}
template CycleVecs<double>& cycle_vecs<double>(Hierarchy&, int);
template CycleVecs<float>& cycle_vecs<float>(Hierarchy&, int);

// Batched forward cycles are captured once (on a private stream, so that the
// caller's stream may be the legacy default stream) and replayed on `s`; the
// cycle holds no memset or allocation, only kernel launches on fixed
// buffers.  The per-launch kernel timer needs the eager path.
template <typename T, int NV>
void vcycle(Hierarchy& H, bool transpose, hipStream_t s) {
  CycleVecs<T>& cv = cycle_vecs<T>(H, NV);
  if (NV > 2 && H.graphs && !transpose && !H.timer) {
    GraphCache& gc = *H.graphs;
    const int key = (int)sizeof(T) * 1000 + NV;
    hipGraphExec_t e = gc.find(key);
    if (!e) {
      if (!gc.cap) FPC_HIP(hipStreamCreateWithFlags(&gc.cap, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      FPC_HIP(hipStreamBeginCapture(gc.cap, hipStreamCaptureModeThreadLocal));
      try {
        vcycle_rec<T, NV>(H, cv, 0, false, gc.cap);
      } catch (...) {
        (void)hipStreamEndCapture(gc.cap, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      FPC_HIP(hipStreamEndCapture(gc.cap, &g));
      const hipError_t ie = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        FPC_HIP(ie);
      }
      gc.slots.push_back({key, g, e});
    }
    FPC_HIP(hipGraphLaunch(e, s));
    return;
  }
  vcycle_rec<T, NV>(H, cv, 0, transpose, s);
}

template <typename T>
void vcycle_to(Hierarchy& H, bool transpose, bool d0_ready, double* out,
               hipStream_t s) {
  CycleVecs<T>& cv = cycle_vecs<T>(H, 1);
  if (H.L.empty() || H.L[0].coarsest) {
    vcycle_rec<T, 1>(H, cv, 0, transpose, s);
    from_level<T>(cv.lv[0].xo.p, 1, H.L.empty() ? 0 : H.nc, out, 0, s);
    return;
  }
  vcycle_rec<T, 1>(H, cv, 0, transpose, s, CycleEnds{d0_ready, out});
}
template void vcycle_to<double>(Hierarchy&, bool, bool, double*, hipStream_t);
template void vcycle_to<float>(Hierarchy&, bool, bool, double*, hipStream_t);

template void vcycle<double, 1>(Hierarchy&, bool, hipStream_t);
template void vcycle<float, 1>(Hierarchy&, bool, hipStream_t);
template void vcycle<double, 8>(Hierarchy&, bool, hipStream_t);
template void vcycle<double, 32>(Hierarchy&, bool, hipStream_t);
template void vcycle<float, 8>(Hierarchy&, bool, hipStream_t);
template void vcycle<float, 32>(Hierarchy&, bool, hipStream_t);

void sell_mv_b(const Sell<double>& A, const double* x, double* y, int KB,
               hipStream_t s) {
  if (A.br != 3 || A.bc != 3) throw Error(FPC_ERR_ARG, "sell_mv_b shape");
  if (KB == 8)
    launch_sell<double, 3, 3, 8>(A, LoadX<double, 8>{x},
                                 EpiStore<double, 8>{y}, s);
  else if (KB == 32)
    launch_sell<double, 3, 3, 32>(A, LoadX<double, 32>{x},
                                  EpiStore<double, 32>{y}, s);
  else
    throw Error(FPC_ERR_ARG, "sell_mv_b: batch width");
}

void sell_mv(const Sell<double>& A, const double* x, double* y, hipStream_t s) {
  if (A.br == 3 && A.bc == 3)
    launch_sell<double, 3, 3, 1>(A, LoadX<double, 1>{x},
                                 EpiStore<double, 1>{y}, s);
  else if (A.br == 6 && A.bc == 6)
    launch_sell<double, 6, 6, 1>(A, LoadX<double, 1>{x},
                                 EpiStore<double, 1>{y}, s);
  else
    throw Error(FPC_ERR_ARG, "sell_mv: unsupported block shape");
}

void sell_mv_dinv(const Sell<double>& A, const double* dinv, const double* x,
                  double* y, hipStream_t s) {
  if (A.br == 3 && A.bc == 3)
    launch_sell<double, 3, 3, 1>(A, LoadX<double, 1>{x},
                                 EpiDinv<double, 1>{dinv, y}, s);
  else if (A.br == 6 && A.bc == 6)
    launch_sell<double, 6, 6, 1>(A, LoadX<double, 1>{x},
                                 EpiDinv<double, 1>{dinv, y}, s);
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
struct LevelPrep {
  T* d0 = nullptr;          // first Chebyshev direction of the finest level
  const T* dinv = nullptr;
  T inv_theta = T(0);
};

// to_level; with prep.d0, also the finest level's first Chebyshev direction
// (formed only on the row-list path: returns whether it was)
template <typename T>
bool to_level_impl(T* out, int nv, int colv, int64_t n, const double* base,
                   const Csr* m1, const double* x1, double a1, const Csr* m2,
                   const double* x2, double a2, const LevelPrep<T>& prep,
                   hipStream_t s) {
  if (n == 0) return prep.d0 != nullptr;
  if (m1 && m1->nact >= 0 && (!m2 || m2->nact >= 0)) {
    // base everywhere, then the rows the coupling blocks touch
    k_base_copy<T><<<grid_for(n, 256), 256, 0, s>>>(out, nv, colv, base, n,
                                                     prep.d0, prep.dinv,
                                                     prep.inv_theta);
    const int64_t* rp2 = m2 ? m2->rowptr.p : nullptr;
    const int64_t nr2 = m2 ? m2->nact : 0;
    if (m1->nact + nr2 > 0)
      k_to_level_rows<T><<<grid_for(m1->nact + nr2, 256), 256, 0, s>>>(
          out, nv, colv, base, m1->act.p, m1->nact,
          m2 ? m2->act.p : nullptr, nr2, m1->rowptr.p, m1->col.p, m1->val.p,
          x1, a1, rp2, m2 ? m2->col.p : nullptr, m2 ? m2->val.p : nullptr,
          x2, a2, prep.d0, prep.dinv, prep.inv_theta);
    FPC_LAUNCH_CHECK();
    return prep.d0 != nullptr;
  }
  k_to_level<T><<<grid_for(n, 256), 256, 0, s>>>(
      out, nv, colv, base, m1 ? m1->rowptr.p : nullptr,
      m1 ? m1->col.p : nullptr, m1 ? m1->val.p : nullptr, x1, a1,
      m2 ? m2->rowptr.p : nullptr, m2 ? m2->col.p : nullptr,
      m2 ? m2->val.p : nullptr, x2, a2, n);
  FPC_LAUNCH_CHECK();
  return false;
}

template <typename T>
void to_level(T* out, int nv, int colv, int64_t n, const double* base,
              const Csr* m1, const double* x1, double a1, const Csr* m2,
              const double* x2, double a2, hipStream_t s) {
  (void)to_level_impl<T>(out, nv, colv, n, base, m1, x1, a1, m2, x2, a2,
                         LevelPrep<T>{}, s);
}

template <typename T>
bool vcycle_input(Hierarchy& H, const double* base, const Csr* m1,
                  const double* x1, double a1, const Csr* m2,
                  const double* x2, double a2, hipStream_t s) {
  CycleVecs<T>& cv = cycle_vecs<T>(H, 1);
  const Level& L = H.L[0];
  LevelPrep<T> prep;
  if (!L.coarsest) {
    prep.d0 = cv.lv[0].d0.p;
    prep.dinv = seldinv<T>(L);
    prep.inv_theta = T(1.0 / L.theta);
  }
  return to_level_impl<T>(cv.lv[0].b.p, 1, 0, L.n_nodes * L.bs, base, m1, x1,
                          a1, m2, x2, a2, prep, s);
}
template bool vcycle_input<double>(Hierarchy&, const double*, const Csr*,
                                   const double*, double, const Csr*,
                                   const double*, double, hipStream_t);
template bool vcycle_input<float>(Hierarchy&, const double*, const Csr*,
                                  const double*, double, const Csr*,
                                  const double*, double, hipStream_t);
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
  k_tface<<<(unsigned)((n_p + 63) / 64), 192, 0, s>>>(C.rowptr.p, C.col.p,
                                                     C.val.p, vu, t_t, hinv,
                                                     v_t, n_p, trans);
  FPC_LAUNCH_CHECK();
}

}  // namespace fpc
