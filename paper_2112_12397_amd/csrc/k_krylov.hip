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

__global__ void k_gmres_step(double* H, int ldh, double* cs, double* sn,
                             double* g, const double* h1, const double* h2,
                             const double* nrm2, const double* nrm2_before,
                             int j, double* scal, int* ctrl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double col[kMaxKrylov + 1];
  for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
  const double hn = sqrt(fmax(nrm2[0], 0.0));
  const double w0 = sqrt(fmax(nrm2_before[0], 0.0));
  col[j + 1] = hn;
  const int breakdown = !(hn > 1e-14 * w0);
  scal[0] = breakdown ? 0.0 : hn;
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double rho = hypot(col[j], col[j + 1]);
  const double c = rho != 0.0 ? col[j] / rho : 1.0;
  const double sgn = rho != 0.0 ? col[j + 1] / rho : 0.0;
  cs[j] = c;
  sn[j] = sgn;
  col[j] = rho;
  col[j + 1] = 0.0;
  g[j + 1] = -sgn * g[j];
  g[j] = c * g[j];
  for (int i = 0; i <= j + 1; ++i) H[(int64_t)i * ldh + j] = col[i];
  scal[1] = fabs(g[j + 1]);
  ctrl[0] = breakdown;
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

int64_t mdot_partials(int64_t n, int nv) {
  return (int64_t)nv * std::max<int64_t>((n + DT * MR - 1) / (DT * MR), 1);
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
