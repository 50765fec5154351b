// Transmissibility gradient of a loss through the adjoint pressure
// (dL/d log Upsilon_K = -lam_p^T (dT/d log Upsilon_K) p, with T the TPFA
// matrix of eq. FV_inner_product: harmonic averages on face pairs plus the
// Dirichlet edges of a face).
//
// The face pairs arrive as two index arrays.  A face's incident pairs are
// listed through a small int32 work area (counts, offsets, pair lists), so
// that every face sums its terms in ascending pair order: the result does
// not depend on scheduling.  Every pair is validated before any index is
// used to address a face array.
#include "fpc_internal.hpp"

namespace fpc {

namespace {

constexpr int kScanT = 1024;

__global__ void k_grad_zero(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Valid pairs (0 <= K, L < n_p, K != L) add one to the count of both faces;
// an invalid pair raises the pattern flag and is skipped.
__global__ void k_grad_count(const int32_t* __restrict__ pk,
                             const int32_t* __restrict__ pl, int64_t m,
                             int64_t n_p, int32_t* cnt, int* flags) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int32_t K = pk[e], L = pl[e];
  if (K < 0 || L < 0 || K >= n_p || L >= n_p || K == L) {
    atomicOr(&flags[FLAG_PATTERN], 1);
    return;
  }
  atomicAdd(&cnt[K], 1);
  atomicAdd(&cnt[L], 1);
}

// off[0] = 0, off[i + 1] = off[i] + cnt[i]: one workgroup, each thread scans
// a contiguous chunk, the chunk totals are scanned in LDS.
__global__ __launch_bounds__(kScanT) void k_grad_scan(
    const int32_t* __restrict__ cnt, int64_t n, int32_t* __restrict__ off) {
  __shared__ int32_t part[kScanT];
  const int t = threadIdx.x;
  const int64_t per = (n + kScanT - 1) / kScanT;
  const int64_t a = t * per, b = a + per < n ? a + per : n;
  int32_t sum = 0;
  for (int64_t i = a; i < b; ++i) sum += cnt[i];
  part[t] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan of the chunk totals
  for (int d = 1; d < kScanT; d <<= 1) {
    const int32_t v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = part[t] - sum;
  if (t == 0) off[0] = 0;
  for (int64_t i = a; i < b; ++i) {
    run += cnt[i];
    off[i + 1] = run;
  }
}

// Pair e enters the lists of K and L (slots taken from the counts, which
// return to zero).  Invalid pairs were flagged and are skipped here too.
__global__ void k_grad_fill(const int32_t* __restrict__ pk,
                            const int32_t* __restrict__ pl, int64_t m,
                            int64_t n_p, const int32_t* __restrict__ off,
                            int32_t* cnt, int32_t* __restrict__ list) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int32_t K = pk[e], L = pl[e];
  if (K < 0 || L < 0 || K >= n_p || L >= n_p || K == L) return;
  list[off[K] + atomicSub(&cnt[K], 1) - 1] = (int32_t)e;
  list[off[L] + atomicSub(&cnt[L], 1) - 1] = (int32_t)e;
}

// Face K: its pair list sorted ascending (insertion sort of a short list),
// then -sum_e dT_KL/dlogU_K (lam_K - lam_L)(p_K - p_L) with the harmonic
// average U_KL = 2 U_K U_L / (U_K + U_L), minus the Dirichlet term
// ndir_K U_K lam_K p_K.
__global__ void k_grad_face(const int32_t* __restrict__ off,
                            int32_t* __restrict__ list,
                            const int32_t* __restrict__ pk,
                            const int32_t* __restrict__ pl,
                            const int32_t* __restrict__ ndir,
                            const double* __restrict__ ups,
                            const double* __restrict__ lam,
                            const double* __restrict__ p, double* grad,
                            int64_t n_p) {
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= n_p) return;
  const int32_t a = off[K], b = off[K + 1];
  for (int32_t i = a + 1; i < b; ++i) {
    const int32_t v = list[i];
    int32_t j = i - 1;
    while (j >= a && list[j] > v) {
      list[j + 1] = list[j];
      --j;
    }
    list[j + 1] = v;
  }
  double g = 0.0;
  for (int32_t q = a; q < b; ++q) {
    const int32_t e = list[q];
    const int32_t L = (pk[e] == K) ? pl[e] : pk[e];
    const double uK = ups[K], uL = ups[L];
    const double s = uK + uL;
    const double dK = 2.0 * uK * uL * uL / (s * s);
    g -= dK * (lam[K] - lam[L]) * (p[K] - p[L]);
  }
  g -= (double)ndir[K] * ups[K] * lam[K] * p[K];
  grad[K] = g;
}

}  // namespace

int64_t grad_scratch_words(int64_t n_p, int64_t n_pairs) {
  return 2 * n_p + 1 + 2 * n_pairs;
}

void grad_validate(int64_t n_p, int64_t n_pairs, const int32_t* pair_k,
                   const int32_t* pair_l, int32_t* work, int* flags,
                   hipStream_t s) {
  int32_t* cnt = work;
  k_grad_zero<<<grid_for(n_p, 256), 256, 0, s>>>(cnt, n_p);
  FPC_LAUNCH_CHECK();
  if (n_pairs > 0) {
    k_grad_count<<<grid_for(n_pairs, 256), 256, 0, s>>>(pair_k, pair_l,
                                                        n_pairs, n_p, cnt,
                                                        flags);
    FPC_LAUNCH_CHECK();
  }
}

void grad_finish(int64_t n_p, int64_t n_pairs, const int32_t* pair_k,
                 const int32_t* pair_l, const int32_t* ndir,
                 const double* upsilon, const double* lam_p, const double* p,
                 double* grad, int32_t* work, hipStream_t s) {
  int32_t* cnt = work;
  int32_t* off = work + n_p;
  int32_t* list = work + 2 * n_p + 1;
  k_grad_scan<<<1, kScanT, 0, s>>>(cnt, n_p, off);
  FPC_LAUNCH_CHECK();
  if (n_pairs > 0) {
    k_grad_fill<<<grid_for(n_pairs, 256), 256, 0, s>>>(pair_k, pair_l, n_pairs,
                                                       n_p, off, cnt, list);
    FPC_LAUNCH_CHECK();
  }
  k_grad_face<<<grid_for(n_p, 256), 256, 0, s>>>(off, list, pair_k, pair_l,
                                                 ndir, upsilon, lam_p, p, grad,
                                                 n_p);
  FPC_LAUNCH_CHECK();
}

}  // namespace fpc
