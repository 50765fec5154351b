// C ABI of the fracprec library: setup of the block preconditioner
// (Alg 3.1 / 3.3) with the smoothed-aggregation hierarchy, its application
// (Alg 3.2 / 3.4) and transpose, the Jacobian product, and right-
// preconditioned FGMRES for one, several or transposed systems.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <atomic>
#include <mutex>
#include <string>

#include "fpc_apply.hpp"

using namespace fpc;

namespace {

double now_s() {
  return std::chrono::duration<double>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// ------------------------------------------------------------- kernels
__global__ void k_dense_transpose(const double* A, double* T, int64_t n) {
  __shared__ double t[32][33];
  int64_t bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += 8) {
    int64_t r = by + k, c = bx + threadIdx.x;
    if (r < n && c < n) t[k][threadIdx.x] = A[r * n + c];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += 8) {
    int64_t r = bx + k, c = by + threadIdx.x;
    if (r < n && c < n) T[r * n + c] = t[threadIdx.x][k];
  }
}

__global__ void k_copy_i32(const int32_t* a, int32_t* b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ void k_cast_dinv(const double* a, float* b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ------------------------------------------------------------- helpers
void check_flags(fpc_handle* h, const char* where) {
  int f[FLAG_COUNT];
  FPC_HIP(hipMemcpyAsync(f, h->flags.p, sizeof(f), hipMemcpyDeviceToHost,
                         h->stream));
  FPC_HIP(hipStreamSynchronize(h->stream));
  std::string w(where);
  if (f[FLAG_PATTERN]) throw Error(FPC_ERR_PATTERN, w + ": invalid CSR pattern");
  if (f[FLAG_NAN]) throw Error(FPC_ERR_NAN, w + ": non-finite value");
  if (f[FLAG_SINGULAR]) throw Error(FPC_ERR_SINGULAR_BLOCK, w + ": singular block or pivot");
  if (f[FLAG_NOT_SPD]) throw Error(FPC_ERR_NOT_SPD, w + ": nonpositive pivot");
  if (f[FLAG_OVERFLOW]) throw Error(FPC_ERR_UNSUPPORTED, w + ": SpGEMM row too long");
}

void upload_csr(const fpc_csr& in, int space, int64_t nr, int64_t nc, Csr& out,
                hipStream_t s, const char* name) {
  if (in.nrows != nr || in.ncols != nc)
    throw Error(FPC_ERR_DIM, std::string(name) + ": shape mismatch");
  if (in.nnz < 0 || !in.rowptr || (in.nnz > 0 && (!in.colind || !in.val)))
    throw Error(FPC_ERR_ARG, std::string(name) + ": null array");
  out.nrows = nr;
  out.ncols = nc;
  out.nnz = in.nnz;
  out.rowptr.alloc(nr + 1);
  out.col.alloc(std::max<int64_t>(in.nnz, 1));
  out.val.alloc(std::max<int64_t>(in.nnz, 1));
  const hipMemcpyKind k =
      space == FPC_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  FPC_HIP(hipMemcpyAsync(out.rowptr.p, in.rowptr, (nr + 1) * sizeof(int64_t), k, s));
  if (in.nnz) {
    FPC_HIP(hipMemcpyAsync(out.col.p, in.colind, in.nnz * sizeof(int32_t), k, s));
    FPC_HIP(hipMemcpyAsync(out.val.p, in.val, in.nnz * sizeof(double), k, s));
  }
}

template <typename F>
fpc_status guard(fpc_handle* h, F&& f) {
  StreamScope scope(h ? h->stream : nullptr);
  try {
    f();
    return FPC_OK;
  } catch (const Error& e) {
    if (h) h->last_error = e.what();
    return e.st;
  } catch (const std::exception& e) {
    if (h) h->last_error = e.what();
    return FPC_ERR_HIP;
  }
}

int64_t round64(int64_t n) { return ((n + 63) / 64) * 64; }

// ------------------------------------------------------------- p-block
// Exact solve of S~2 = T - FS(Q2, S1, Q1) (T - diag(S_K) in t-u-p and M2*
// with open faces, T otherwise): nested-dissection ordering and symbolic
// analysis of T's pattern, then the multifrontal factorization.  With
// `reuse` (numeric re-setup), a matrix with the pattern of the previous
// factorization keeps its analysis, and one with the same values too keeps
// the factor; without it everything is built.
void build_psolve(fpc_handle* h, bool reuse) {
  PSolve& ps = h->ps;
  const int64_t n = h->n_p;
  hipStream_t s = h->stream;
  const Csr& T = h->T;
  const bool fs = h->opt.mode != FPC_TPU && h->has_q2;
  const double* sk = fs ? h->S_K.p : nullptr;
  if (n == 0) {
    ps = PSolve();
    return;
  }
  const bool same_pat =
      reuse && ps.n == n &&
      ps.in_col.n == (size_t)std::max<int64_t>(T.nnz, 1) &&
      same_pattern(ps.in_rp.p, ps.in_col.p, T.rowptr.p, T.col.p, n, T.nnz, s);
  if (same_pat && ps.in_val.p && ps.has_sk == fs &&
      same_values(ps.in_val.p, T.val.p, T.nnz, s) &&
      (!fs || (ps.in_sk.p && same_values(ps.in_sk.p, sk, n, s))))
    return;  // the factor of this matrix is in place
  ps.in_val.release();  // no factor is valid until this one completes
  if (!same_pat) {
    fill_i32(h->flags.p, 0, FLAG_COUNT, s);
    psolve_analyse(ps, T, h->flags.p, s);
    check_flags(h, "pressure block (nested dissection of a symmetric S~2)");
    ps.in_rp.alloc(n + 1);
    ps.in_col.alloc(std::max<int64_t>(T.nnz, 1));
    FPC_HIP(hipMemcpyAsync(ps.in_rp.p, T.rowptr.p, (n + 1) * sizeof(int64_t),
                           hipMemcpyDeviceToDevice, s));
    if (T.nnz)
      FPC_HIP(hipMemcpyAsync(ps.in_col.p, T.col.p, T.nnz * sizeof(int32_t),
                             hipMemcpyDeviceToDevice, s));
  }
  fill_i32(h->flags.p, 0, FLAG_COUNT, s);
  psolve_factor(ps, T, sk, /*spd=*/!fs, h->flags.p, s);
  check_flags(h, "pressure block factorization");
  ps.in_val.alloc(std::max<int64_t>(T.nnz, 1));
  if (T.nnz)
    FPC_HIP(hipMemcpyAsync(ps.in_val.p, T.val.p, T.nnz * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  ps.has_sk = fs;
  if (fs) {
    ps.in_sk.alloc(n);
    FPC_HIP(hipMemcpyAsync(ps.in_sk.p, sk, n * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  } else {
    ps.in_sk.release();
  }
  FPC_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------- AMG setup
double power_lambda(fpc_handle* h, Level& L, int key_stride) {
  hipStream_t s = h->stream;
  const int64_t n = L.n_nodes * L.bs;
  DevBuf<double> x(n), y(n), part(kRedBlocks), sc(2);
  power_start(L.n_nodes, L.bs, key_stride,
              L.node_rank.p ? L.node_rank.p : nullptr, x.p, s);
  dot_f64(x.p, x.p, n, sc.p, part.p, s);
  sqrt_dev(sc.p, sc.p + 1, s);
  scale_by_inv(x.p, sc.p + 1, x.p, n, s);
  for (int it = 0; it < h->opt.amg.power_its; ++it) {
    sell_mv_dinv(L.sA, L.dinv.p, x.p, y.p, s);
    dot_f64(y.p, y.p, n, sc.p, part.p, s);
    sqrt_dev(sc.p, sc.p + 1, s);
    scale_by_inv(y.p, sc.p + 1, x.p, n, s);
  }
  return read_f64(sc.p + 1, s);
}

// With `prev` (a hierarchy built on the same level-0 block pattern), the
// pattern-only parts are taken over instead of recomputed: the aggregates
// (structure-only MIS-2), the tentative prolongators and coarse ranks (they
// depend on the aggregates and the coordinates only), the apply layouts, the
// patterns of the Galerkin products and the transpose plan of R.
// Everything that depends on values is recomputed, so the result equals a
// fresh build.
void build_hierarchy(fpc_handle* h, Bsr&& S1, Hierarchy* prev = nullptr) {
  Hierarchy& H = h->amg;
  h->graphs.clear();  // captured cycles refer to the old hierarchy
  H = Hierarchy();
  H.timer = h->ktimer.on ? &h->ktimer : nullptr;
  H.graphs = h->opt.graphs ? &h->graphs : nullptr;
  hipStream_t s = h->stream;
  const fpc_amg_options& o = h->opt.amg;
  const int nb = h->has_coords ? 6 : 3;
  H.L.emplace_back();
  {
    Level& L0 = H.L.back();
    L0.bs = 3;
    L0.A = std::move(S1);
    L0.n_nodes = L0.A.nbr;
    L0.n_dofs_real = 3 * L0.n_nodes;
  }
  DevBuf<double> B;
  if (!prev) {
    B.alloc(H.L[0].n_nodes * 3 * nb);
    rigid_modes(h->has_coords ? h->coords.p : nullptr, H.L[0].n_nodes, nb, B.p,
                s);
  }
  while (true) {
    Level& L = H.L.back();
    const size_t li = H.L.size() - 1;
    Level* pv = prev && li < prev->L.size() ? &prev->L[li] : nullptr;
    if (prev && !pv) throw Error(FPC_ERR_STATE, "re-setup: level count changed");
    L.dinv.alloc(L.n_nodes * L.bs);
    bsr_dinv(L.A, L.dinv.p, h->flags.p, s);
    check_flags(h, "AMG diagonal");
    if (L.n_dofs_real <= o.max_coarse || (int)H.L.size() == o.max_levels) {
      L.coarsest = true;
      break;
    }
    if (pv) {
      if (pv->coarsest || pv->n_nodes != L.n_nodes)
        throw Error(FPC_ERR_STATE, "re-setup: hierarchy shape changed");
      L.agg = std::move(pv->agg);
      L.n_agg = pv->n_agg;
    } else {
      L.agg.alloc(L.n_nodes);
      DevBuf<int32_t> roots;
      L.n_agg = aggregate_mis2(L.A, L.agg.p, roots, s);
    }
    if (L.n_agg == 0) {
      L.coarsest = true;
      break;
    }
    L.nb = nb;
    bsr_to_sell(L.A, L.sA, s);
    const double lam = power_lambda(h, L, L.bs);
    L.lam_hi = o.lam_safety * lam;
    const double lo = L.lam_hi / o.cheb_ratio;
    L.theta = 0.5 * (L.lam_hi + lo);
    L.delta = 0.5 * (L.lam_hi - lo);
    const double sigma = L.theta / L.delta;
    const double rho0 = 1.0 / sigma;
    const double rho1 = 1.0 / (2.0 * sigma - rho0);
    L.c1 = rho1 * rho0;
    L.c2 = 2.0 * rho1 / L.delta;
    // tentative prolongator
    DevBuf<double> Bc;
    if (pv) {
      L.rank = std::move(pv->rank);
      L.Pt = std::move(pv->Pt);
    } else {
      DevBuf<double> ptent(L.n_nodes * L.bs * nb);
      Bc.alloc(L.n_agg * nb * nb);
      L.rank.alloc(L.n_agg);
      tentative(L.agg.p, L.n_nodes, L.n_agg, L.bs, nb, B.p, o.drop_tol,
                ptent.p, Bc.p, L.rank.p, s);
      ptent_bsr(L.agg.p, L.n_nodes, L.n_agg, L.bs, nb, ptent.p, L.Pt, s);
    }
    // the products' patterns follow from the operands' patterns, which a
    // re-setup keeps: only their numeric phases run then
    Bsr AP0;
    spgemm(L.A, L.Pt, AP0, h->flags.p, s, /*b_single=*/true, &L.pat_ap0,
           pv ? &pv->pat_ap0 : nullptr);
    // P = P_tent - omega D^{-1} (A P_tent)
    smooth_prolongator(AP0, L.dinv.p, o.omega_factor / L.lam_hi, s);
    bsr_add(L.Pt, AP0, L.P, s);
    bsr_transpose(L.P, L.R, s, &L.plan_r, pv ? &pv->plan_r : nullptr);
    Bsr AP, Ac;
    spgemm(L.A, L.P, AP, h->flags.p, s, false, &L.pat_ap,
           pv ? &pv->pat_ap : nullptr);
    spgemm(L.R, AP, Ac, h->flags.p, s, false, &L.pat_ac,
           pv ? &pv->pat_ac : nullptr);
    check_flags(h, "Galerkin product");
    dummy_diag(Ac, L.rank.p, s);
    // next level
    std::vector<int32_t> rk(L.n_agg);
    FPC_HIP(hipMemcpyAsync(rk.data(), L.rank.p, L.n_agg * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
    FPC_HIP(hipStreamSynchronize(s));
    int64_t real = 0;
    for (int32_t r : rk) real += r;
    const int64_t n_agg = L.n_agg;
    Level next;
    next.bs = nb;
    next.A = std::move(Ac);
    next.n_nodes = n_agg;
    next.n_dofs_real = real;
    next.node_rank.alloc(n_agg);
    k_copy_i32<<<grid_for(n_agg, 256), 256, 0, s>>>(L.rank.p, next.node_rank.p,
                                                    n_agg);
    FPC_LAUNCH_CHECK();
    if (!pv) B = std::move(Bc);
    H.L.push_back(std::move(next));
  }
  // coarsest level: dense inverse (FP64)
  Level& C = H.L.back();
  H.nc = C.n_nodes * C.bs;
  H.ncpad = round64(std::max<int64_t>(H.nc, 1));
  H.Ainv.alloc(H.ncpad * H.ncpad);
  dense_from_bsr(C.A, H.ncpad, H.Ainv.p, s);
  gj_inverse(H.Ainv.p, H.ncpad, h->flags.p, s);
  check_flags(h, "coarsest level");
  // apply layouts, tuned for the column count of the preconditioner
  const int nv = 1;
  for (size_t li = 0; li < H.L.size(); ++li) {
    Level& L = H.L[li];
    if (L.coarsest) continue;
    // L.sA (built for the power iteration) is handed to the FP64 layout
    // choice and released otherwise
    if (prev || h->opt.tune != 1) {
      // the layouts picked for the same patterns, or by the shape alone
      const Bsr* ops[3] = {&L.A, &L.P, &L.R};
      for (int k = 0; k < 3; ++k) {
        L.layout[k] = prev ? prev->L[li].layout[k]
                           : rule_layout(*ops[k], h->opt.tune == 2);
        L.tune_us[k] = prev ? prev->L[li].tune_us[k] : 0.0;
      }
      if (h->opt.precision == FPC_FP32_PREC) {
        const int64_t n = L.n_nodes * L.bs;
        L.dinv32.alloc(n);
        k_cast_dinv<<<grid_for(n, 256), 256, 0, s>>>(L.dinv.p, L.dinv32.p, n);
        FPC_LAUNCH_CHECK();
        build_op<float>(L.A, L.layout[0], L.fA, s);
        build_op<float>(L.P, L.layout[1], L.fP, s);
        build_op<float>(L.R, L.layout[2], L.fR, s);
      } else {
        build_op<double>(L.A, L.layout[0], L.oA, s, &L.sA);
        build_op<double>(L.P, L.layout[1], L.oP, s);
        build_op<double>(L.R, L.layout[2], L.oR, s);
      }
      L.sA = Sell<double>();
      continue;
    }
    if (h->opt.precision == FPC_FP32_PREC) {
      const int64_t n = L.n_nodes * L.bs;
      L.dinv32.alloc(n);
      k_cast_dinv<<<grid_for(n, 256), 256, 0, s>>>(L.dinv.p, L.dinv32.p, n);
      FPC_LAUNCH_CHECK();
      tune_op<float>(L.A, nv, L.fA, s, &L.layout[0],
                      &L.tune_us[0]);
      tune_op<float>(L.P, nv, L.fP, s, &L.layout[1],
                      &L.tune_us[1]);
      tune_op<float>(L.R, nv, L.fR, s, &L.layout[2],
                      &L.tune_us[2]);
    } else {
      tune_op<double>(L.A, nv, L.oA, s, &L.layout[0],
                      &L.tune_us[0], &L.sA);
      tune_op<double>(L.P, nv, L.oP, s, &L.layout[1],
                      &L.tune_us[1]);
      tune_op<double>(L.R, nv, L.oR, s, &L.layout[2],
                      &L.tune_us[2]);
    }
    L.sA = Sell<double>();
  }
  FPC_HIP(hipStreamSynchronize(s));
}

void ensure_transposes(fpc_handle* h) {
  if (h->have_T) return;
  hipStream_t s = h->stream;
  csr_transpose(h->C1, h->C1T, s);
  csr_transpose(h->C2, h->C2T, s);
  csr_transpose(h->Q1, h->Q1T, s);
  csr_transpose(h->Q2, h->Q2T, s);
  csr_active_rows(h->C2T, s);
  csr_active_rows(h->Q2T, s);
  csr_transpose(h->H, h->HT, s);
  csr_transpose(h->T, h->TT, s);
  Bsr AbT;
  bsr_transpose(h->Ab, AbT, s);
  bsr_to_sell(AbT, h->sAJT, s);
  Hierarchy& H = h->amg;
  for (Level& L : H.L) {
    if (L.coarsest) continue;
    bsr_transpose(L.A, L.AT, s);
    const bool f32 = h->opt.precision == FPC_FP32_PREC;
    const bool timed = h->opt.tune == 1;
    const int rule = rule_layout(L.AT, h->opt.tune == 2);
    if (!timed && f32) build_op<float>(L.AT, rule, L.fAT, s);
    else if (!timed) build_op<double>(L.AT, rule, L.oAT, s);
    else if (f32) tune_op<float>(L.AT, 1, L.fAT, s, nullptr, nullptr);
    else tune_op<double>(L.AT, 1, L.oAT, s, nullptr, nullptr);
  }
  H.AinvT.alloc(H.ncpad * H.ncpad);
  dim3 g((unsigned)((H.ncpad + 31) / 32), (unsigned)((H.ncpad + 31) / 32));
  k_dense_transpose<<<g, dim3(32, 8), 0, s>>>(H.Ainv.p, H.AinvT.p, H.ncpad);
  FPC_LAUNCH_CHECK();
  FPC_HIP(hipStreamSynchronize(s));
  h->have_T = true;
}

// ------------------------------------------------------------- apply
void matvec(fpc_handle* h, int trans, const double* x, double* y) {
  hipStream_t s = h->stream;
  const double *xu = x, *xt = x + h->n_u, *xp = x + h->n_u + h->n_t;
  double *yu = y, *yt = y + h->n_u, *yp = y + h->n_u + h->n_t;
  // the A block, then the coupling rows of y_u and the t and p rows in one
  // launch
  if (!trans) {
    sell_mv(h->sAJ, xu, yu, s);
    csr_spmv2_many({{&h->C1, xt, 1.0, &h->Q1, xp, 1.0, yu, 1.0},
                    {&h->C2, xu, 1.0, &h->H, xt, -1.0, yt, 0.0},
                    {&h->Q2, xu, 1.0, &h->T, xp, 1.0, yp, 0.0}},
                   s);
  } else {
    ensure_transposes(h);
    sell_mv(h->sAJT, xu, yu, s);
    csr_spmv2_many({{&h->C2T, xt, 1.0, &h->Q2T, xp, 1.0, yu, 1.0},
                    {&h->C1T, xu, 1.0, &h->HT, xt, -1.0, yt, 0.0},
                    {&h->Q1T, xu, 1.0, &h->TT, xp, 1.0, yp, 0.0}},
                   s);
  }
}

// Whether the forward application starts with steps that depend on w only
// (t_t = H~^-1 w_t and v_p = S~2^-1 w_p: the Q2 = 0 t-u-p and t-p-u paths),
// so that they may run ahead of the rest.
bool fwd_has_lead(const fpc_handle* h) {
  return !h->has_q2 && (h->opt.mode == FPC_TUP || h->opt.mode == FPC_TPU);
}

// stage 0: the whole application; with fwd_has_lead(h), stage 1 runs the
// leading face and pressure solves only and stage 2 the rest.
template <typename T>
void apply_fwd(fpc_handle* h, const double* w, double* v, int stage = 0) {
  hipStream_t s = h->stream;
  const int64_t nu = h->n_u, nt = h->n_t, np = h->n_p;
  const double *wu = w, *wt = w + nu, *wp = w + nu + nt;
  double *vu = v, *vt = v + nu, *vp = v + nu + nt;
  if (stage != 0 && fwd_has_lead(h)) {
    if (stage == 1) {
      face_apply(h->hinv.p, wt, h->t_t.p, np, 0, s);        // t_t = H~^-1 w_t
      psolve_apply(h->ps, wp, vp, np, 0, s);                // v_p = S~2^-1 w_p
      return;
    }
    const bool d0 = vcycle_input<T>(h->amg, wu, &h->C1, h->t_t.p, 1.0, &h->Q1,
                                    vp, -1.0, s);
    vcycle_to<T>(h->amg, false, d0, vu, s);
    tface(h->C2, vu, h->t_t.p, h->hinv.p, vt, np, 0, s);    // v_t
    return;
  }
  face_apply(h->hinv.p, wt, h->t_t.p, np, 0, s);            // t_t = H~^-1 w_t
  if (h->opt.mode == FPC_TUP_STAR) {
    // M2* = D2^-1 L2^-1 (eq. LDU2): steps 1-5 of Alg 3.4 with v_u = s_u,
    // v_t = -t_t; one AMG call
    CycleVecs<T>& cv = cycle_vecs<T>(h->amg, 1);
    to_level<T>(cv.lv[0].b.p, 1, 0, nu, wu, &h->C1, h->t_t.p, 1.0, nullptr,
                nullptr, 0.0, s);
    vcycle<T, 1>(h->amg, false, s);
    from_level<T>(cv.lv[0].xo.p, 1, nu, vu, 0, s);          // v_u
    if (h->has_q2) {
      FPC_HIP(hipMemcpyAsync(h->tmp_p.p, wp, np * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
      csr_spmv2(&h->Q2, vu, -1.0, nullptr, nullptr, 0.0, h->tmp_p.p, 1.0, s);
      psolve_apply(h->ps, h->tmp_p.p, vp, np, 0, s);
    } else {
      psolve_apply(h->ps, wp, vp, np, 0, s);
    }
    axpby(-1.0, h->t_t.p, 0.0, vt, nt, s);                  // v_t = -t_t
    return;
  }
  if (h->has_q2 && h->opt.mode == FPC_TUP) {
    // Alg 3.4 with open faces: t_p depends on s_u, the AMG calls of steps 3
    // and 7 run one after the other
    CycleVecs<T>& cv = cycle_vecs<T>(h->amg, 1);
    double* su = h->tmp_u.p;
    to_level<T>(cv.lv[0].b.p, 1, 0, nu, wu, &h->C1, h->t_t.p, 1.0, nullptr,
                nullptr, 0.0, s);                            // t_u
    vcycle<T, 1>(h->amg, false, s);
    from_level<T>(cv.lv[0].xo.p, 1, nu, su, 0, s);          // s_u
    FPC_HIP(hipMemcpyAsync(h->tmp_p.p, wp, np * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    csr_spmv2(&h->Q2, su, -1.0, nullptr, nullptr, 0.0, h->tmp_p.p, 1.0, s);
    psolve_apply(h->ps, h->tmp_p.p, vp, np, 0, s);          // v_p = S~2^-1 t_p
    to_level<T>(cv.lv[0].b.p, 1, 0, nu, nullptr, &h->Q1, vp, 1.0, nullptr,
                nullptr, 0.0, s);                            // Q1 v_p
    vcycle<T, 1>(h->amg, false, s);
    from_level<T>(cv.lv[0].xo.p, 1, nu, vu, 0, s);
    axpby(1.0, su, -1.0, vu, nu, s);                        // v_u = s_u - AMG
  } else if (h->has_q2) {
    // Alg 3.2 with open faces: v_p = t_p - T^-1 Q2 v_u
    psolve_apply(h->ps, wp, h->tmp_p.p, np, 0, s);          // t_p = T^-1 w_p
    CycleVecs<T>& cv = cycle_vecs<T>(h->amg, 1);
    to_level<T>(cv.lv[0].b.p, 1, 0, nu, wu, &h->C1, h->t_t.p, 1.0, &h->Q1,
                h->tmp_p.p, -1.0, s);
    vcycle<T, 1>(h->amg, false, s);
    from_level<T>(cv.lv[0].xo.p, 1, nu, vu, 0, s);
    csr_spmv2(&h->Q2, vu, 1.0, nullptr, nullptr, 0.0, h->tmp_p2.p, 0.0, s);
    psolve_apply(h->ps, h->tmp_p2.p, vp, np, 0, s);
    axpby(1.0, h->tmp_p.p, -1.0, vp, np, s);
  } else {
    // Q2 = 0.  Alg 3.4: t_p = w_p, so v_p = S~2^-1 w_p (S~2 = T) is known
    // before the first AMG call, and since the V-cycle is a fixed linear
    // operator the two calls of steps 3 and 7 combine into one:
    // v_u = AMG(t_u) - AMG(Q1 v_p) = AMG(w_u + C1 t_t - Q1 v_p).
    // Alg 3.2: t_p = T^-1 w_p is also v_p, and v_u is the same cycle.
    psolve_apply(h->ps, wp, vp, np, 0, s);
    const bool d0 = vcycle_input<T>(h->amg, wu, &h->C1, h->t_t.p, 1.0, &h->Q1,
                                    vp, -1.0, s);
    vcycle_to<T>(h->amg, false, d0, vu, s);
  }
  tface(h->C2, vu, h->t_t.p, h->hinv.p, vt, np, 0, s);      // v_t
}

template <typename T>
void apply_adj(fpc_handle* h, const double* w, double* v) {
  hipStream_t s = h->stream;
  ensure_transposes(h);
  const int64_t nu = h->n_u, nt = h->n_t, np = h->n_p;
  const double *wu = w, *wt = w + nu, *wp = w + nu + nt;
  double *vu = v, *vt = v + nu, *vp = v + nu + nt;
  // M^{-T}: t_t = H~^-T w_t; t_u = w_u + C2^T t_t; s_u = AMG^T(t_u);
  // t_p = w_p - Q1^T s_u; v_p = S~2^-T t_p; v_u = s_u - AMG^T(Q2^T v_p)
  // (= s_u when Q2 = 0); v_t = -t_t + H~^-T C1^T v_u.  The t-p-u transpose
  // coincides when Q2 = 0.
  face_apply(h->hinv.p, wt, h->t_t.p, np, 1, s);
  CycleVecs<T>& cv = cycle_vecs<T>(h->amg, 1);
  if (h->opt.mode == FPC_TUP_STAR) {
    // M2*^{-T} = L2^-T D2^-T: v_p = S~2^-T w_p; v_u = AMG^T(w_u - Q2^T v_p);
    // v_t = -t_t + H~^-T C1^T v_u
    psolve_apply(h->ps, wp, vp, np, 1, s);
    to_level<T>(cv.lv[0].b.p, 1, 0, nu, wu, h->has_q2 ? &h->Q2T : nullptr, vp,
                -1.0, nullptr, nullptr, 0.0, s);
    vcycle<T, 1>(h->amg, true, s);
    from_level<T>(cv.lv[0].xo.p, 1, nu, vu, 0, s);
    tface(h->C1T, vu, h->t_t.p, h->hinv.p, vt, np, 1, s);
    return;
  }
  if (h->has_q2 && h->opt.mode == FPC_TPU) {
    // M1^{-T} (transposed factors of eq. P1): t_p = T^-T w_p; t_u = w_u +
    // C2^T t_t - Q2^T t_p; v_u = AMG^T(t_u); v_p = t_p - T^-T Q1^T v_u
    psolve_apply(h->ps, wp, h->tmp_p.p, np, 1, s);
    to_level<T>(cv.lv[0].b.p, 1, 0, nu, wu, &h->C2T, h->t_t.p, 1.0, &h->Q2T,
                h->tmp_p.p, -1.0, s);
    vcycle<T, 1>(h->amg, true, s);
    from_level<T>(cv.lv[0].xo.p, 1, nu, vu, 0, s);
    csr_spmv2(&h->Q1T, vu, 1.0, nullptr, nullptr, 0.0, h->tmp_p2.p, 0.0, s);
    psolve_apply(h->ps, h->tmp_p2.p, vp, np, 1, s);
    axpby(1.0, h->tmp_p.p, -1.0, vp, np, s);
    tface(h->C1T, vu, h->t_t.p, h->hinv.p, vt, np, 1, s);
    return;
  }
  to_level<T>(cv.lv[0].b.p, 1, 0, nu, wu, &h->C2T, h->t_t.p, 1.0, nullptr,
              nullptr, 0.0, s);
  vcycle<T, 1>(h->amg, true, s);
  from_level<T>(cv.lv[0].xo.p, 1, nu, vu, 0, s);            // s_u
  FPC_HIP(hipMemcpyAsync(h->tmp_p.p, wp, np * sizeof(double),
                         hipMemcpyDeviceToDevice, s));
  csr_spmv2(&h->Q1T, vu, -1.0, nullptr, nullptr, 0.0, h->tmp_p.p, 1.0, s);
  psolve_apply(h->ps, h->tmp_p.p, vp, np, 1, s);
  if (h->has_q2) {
    // second transposed AMG call on Q2^T v_p
    to_level<T>(cv.lv[0].b.p, 1, 0, nu, nullptr, &h->Q2T, vp, 1.0, nullptr,
                nullptr, 0.0, s);
    vcycle<T, 1>(h->amg, true, s);
    from_level<T>(cv.lv[0].xo.p, 1, nu, h->tmp_u.p, 0, s);
    axpby(-1.0, h->tmp_u.p, 1.0, vu, nu, s);                // v_u = s_u - AMG^T
  }
  tface(h->C1T, vu, h->t_t.p, h->hinv.p, vt, np, 1, s);
}

void apply(fpc_handle* h, int trans, const double* w, double* v,
           int stage = 0) {
  const bool fp32 = h->opt.precision == FPC_FP32_PREC;
  if (!trans) {
    if (fp32) apply_fwd<float>(h, w, v, stage);
    else apply_fwd<double>(h, w, v, stage);
  } else {
    if (fp32) apply_adj<float>(h, w, v);
    else apply_adj<double>(h, w, v);
  }
}

// ------------------------------------------------------------- FGMRES
void ensure_krylov(fpc_handle* h, Krylov& K, int k) {
  const int m = h->opt.restart;
  if (K.m == m && K.k >= k && K.N == h->N) return;
  K.m = m;
  K.k = k;
  K.N = h->N;
  const int64_t N = h->N;
  K.V.alloc((int64_t)(m + 1) * N * k);
  K.Z.alloc((int64_t)m * N * k);
  K.w.alloc(N * k);
  K.r.alloc(N * k);
  K.tmp.alloc(N * k);
  K.H.alloc((int64_t)(m + 1) * m * k);
  K.cs.alloc((int64_t)m * k);
  K.sn.alloc((int64_t)m * k);
  K.g.alloc((int64_t)(m + 1) * k);
  K.y.alloc((int64_t)m * k);
  K.h1.alloc((int64_t)(m + 1) * k);
  K.h2.alloc((int64_t)(m + 1) * k);
  K.scal.alloc(8 * k);
  K.D.alloc(2 * (m + 1) + 1);
  K.P.alloc(m + 1);
  K.partials.alloc(mdot_partials(h->N, 2 * (m + 1) + 1));
  K.ctrl.alloc(4 * k);
  if (!K.host) FPC_HIP(hipHostMalloc((void**)&K.host, 64 * sizeof(double)));
  if (!K.ev) FPC_HIP(hipEventCreateWithFlags(&K.ev, hipEventDisableTiming));
}

double dev_norm(fpc_handle* h, Krylov& K, const double* x, double* slot) {
  mdot(x, 0, 1, x, h->N, K.partials.p, slot, h->stream);
  return std::sqrt(std::max(read_f64(slot, h->stream), 0.0));
}

// One restart cycle of FGMRES with classical Gram-Schmidt twice in three
// passes or modified Gram-Schmidt (u_0 = v_0 = r / beta in slot 0, g = beta
// e_1); returns the number of columns of H.
int cgs_cycle(fpc_handle* h, Krylov& K, int trans, double tol, int& its,
              double& est) {
  hipStream_t s = h->stream;
  const int64_t N = h->N;
  const int m = h->opt.restart;
  double* sc = K.scal.p;
  // The leading steps of M^-1 v_{j+1} (which need v_{j+1} only) are queued
  // before the host waits for the convergence test of step j, so the
  // device has work during that round trip; after the last step of a
  // cycle they are unused.
  const bool lead = !trans && fwd_has_lead(h);
  bool lead_done = false;
  int k = 0;
  for (int j = 0; j < m; ++j) {
    double* vj = K.V.p + (int64_t)j * N;
    double* zj = K.Z.p + (int64_t)j * N;
    if (lead) {
      if (!lead_done) apply(h, trans, vj, zj, 1);
      apply(h, trans, vj, zj, 2);
      lead_done = false;
    } else {
      apply(h, trans, vj, zj);
    }
    matvec(h, trans, zj, K.w.p);
    // |w|^2 before the projections (breakdown test) at nrm_before
    const double* nrm_before = sc + 4;
    if (h->opt.ortho == FPC_MGS) {
      // modified Gram-Schmidt: h_ij = v_i^T w with the w of step i
      mdot(K.w.p, 0, 1, K.w.p, N, K.partials.p, sc + 4, s);
      for (int i = 0; i <= j; ++i) {
        const double* vi = K.V.p + (int64_t)i * N;
        mdot(vi, N, 1, K.w.p, N, K.partials.p, K.h1.p + i, s);
        maxpy(vi, N, 1, K.h1.p + i, K.w.p, N, s);
      }
      FPC_HIP(hipMemsetAsync(K.h2.p, 0, (j + 1) * sizeof(double), s));
      mdot(K.w.p, 0, 1, K.w.p, N, K.partials.p, sc + 5, s);
    } else {
      // classical Gram-Schmidt, twice, in three passes over the basis:
      // h1 = V^T w (and |w|^2); w -= V h1 with h2 = V^T w from the same
      // rows; w -= V h2 with |w|^2
      cgs_dot(K.V.p, N, j + 1, K.w.p, N, K.partials.p, K.h1.p, s);
      nrm_before = K.h1.p + j + 1;
      cgs_axpy_dot(K.V.p, N, j + 1, K.h1.p, K.w.p, N, K.partials.p, K.h2.p,
                   s);
      cgs_axpy_norm(K.V.p, N, j + 1, K.h2.p, K.w.p, N, K.partials.p, sc + 5,
                    s);
    }
    gmres_step(K.H.p, m, K.cs.p, K.sn.p, K.g.p, K.h1.p, K.h2.p, sc + 5,
               nrm_before, j, sc, K.ctrl.p, s);
    // the convergence scalars go to the host ahead of the next vector and
    // its lead stage, and the host waits for them only: the stage-2 work
    // of step j + 1 is queued while the device still runs the lead stage
    FPC_HIP(hipMemcpyAsync(K.host, sc, 8 * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    FPC_HIP(hipEventRecord(K.ev, s));
    scale_by_inv(K.w.p, sc, K.V.p + (int64_t)(j + 1) * N, N, s);
    if (lead && j + 1 < m) {
      apply(h, trans, K.V.p + (int64_t)(j + 1) * N,
            K.Z.p + (int64_t)(j + 1) * N, 1);
      lead_done = true;
    }
    FPC_HIP(hipEventSynchronize(K.ev));
    ++its;
    k = j + 1;
    est = K.host[1];
    const int breakdown = K.host[7] != 0.0;
    if (K.host[1] <= tol || breakdown || its >= h->opt.maxit) break;
  }
  return k;
}

// One restart cycle of FGMRES with the delayed Gram-Schmidt (two passes
// over the basis per step; u_0 = r / beta already in slot 0 and g = beta
// e_1).  Column j of H is made final at step j + 1; the host decides from
// the provisional estimate of column j and, when that one meets the
// tolerance (or the cycle or the iteration budget ends), makes the column
// final with one more dot pass over V_0 .. V_j, u_{j+1} before it stops.
// Returns the number of final columns.
int dcgs2_cycle(fpc_handle* h, Krylov& K, int trans, double tol, int& its,
                double& est) {
  hipStream_t s = h->stream;
  const int64_t N = h->N;
  const int m = h->opt.restart;
  double* sc = K.scal.p;
  // scal: [0] rho_j, [1] provisional estimate, [5] estimate of the last
  // final column, [6] |w|^2 before the projections, [7] the step's code
  // (1: breakdown at step j, 2: rho_j = 0); leading stage of
  // M^-1 u_{j+1} queued before the host waits, as in cgs_cycle
  const bool lead = !trans && fwd_has_lead(h);
  bool lead_done = false;
  bool prev_final = true;  // column j - 1 already final (none for j = 0)
  auto fetch = [&]() {
    FPC_HIP(hipMemcpyAsync(K.host, sc, 8 * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    FPC_HIP(hipEventRecord(K.ev, s));
  };
  for (int j = 0; j < m; ++j) {
    double* uj = K.V.p + (int64_t)j * N;
    double* zj = K.Z.p + (int64_t)j * N;
    if (lead) {
      if (!lead_done) apply(h, trans, uj, zj, 1);
      apply(h, trans, uj, zj, 2);
      lead_done = false;
    } else {
      apply(h, trans, uj, zj);
    }
    matvec(h, trans, zj, K.w.p);
    dcgs_dot(K.V.p, N, j + 1, uj, K.w.p, N, K.partials.p, K.D.p, s);
    dcgs_finish(K.D.p, j + 1, !prev_final, true, K.H.p, m, K.cs.p, K.sn.p,
                K.g.p, K.P.p, sc, K.ctrl.p, s);
    dcgs_update(K.V.p, N, j, K.D.p, K.P.p, sc, K.w.p, N, K.partials.p, s);
    dcgs_peek(K.partials.p, N, K.H.p, m, K.cs.p, K.sn.p, K.g.p, K.P.p, j, sc,
              K.ctrl.p, s);
    fetch();
    if (lead && j + 1 < m) {
      apply(h, trans, K.V.p + (int64_t)(j + 1) * N,
            K.Z.p + (int64_t)(j + 1) * N, 1);
      lead_done = true;
    }
    FPC_HIP(hipEventSynchronize(K.ev));
    ++its;
    const int ctrl = (int)K.host[7];
    if (ctrl == 2) {  // u_j inside span(V_0 .. V_{j-1}): column j - 1 final
      est = K.host[5];
      return j;
    }
    if (ctrl == 1) {  // breakdown at step j: column j committed as it is
      est = K.host[5];
      return j + 1;
    }
    prev_final = false;
    const bool last = j + 1 == m || its >= h->opt.maxit;
    if (j > 0 && K.host[5] <= tol) {
      // column j - 1 (final) already meets the tolerance
      est = K.host[5];
      return j;
    }
    if (K.host[1] <= tol || last) {
      dcgs_dot(K.V.p, N, j + 2, K.V.p + (int64_t)(j + 1) * N, nullptr, N,
               K.partials.p, K.D.p, s);
      dcgs_finish(K.D.p, j + 2, true, false, K.H.p, m, K.cs.p, K.sn.p, K.g.p,
                  K.P.p, sc, K.ctrl.p, s);
      fetch();
      FPC_HIP(hipEventSynchronize(K.ev));
      prev_final = true;
      est = K.host[5];
      if (K.host[5] <= tol || last || K.host[7] == 2.0) return j + 1;
    } else {
      est = K.host[1];
    }
  }
  return m;
}

fpc_status fgmres(fpc_handle* h, int trans, const double* b, double* x,
                  double rtol, int use_x0, fpc_info* info) {
  const double t0 = now_s();
  hipStream_t s = h->stream;
  Krylov& K = h->kry1;
  ensure_krylov(h, K, 1);
  const int64_t N = h->N;
  const int m = h->opt.restart;
  if (rtol <= 0) rtol = h->opt.rtol;
  fill_i32(h->flags.p, 0, FLAG_COUNT, s);
  check_finite(b, N, h->flags.p, s);
  check_flags(h, "right-hand side");
  double* sc = K.scal.p;  // [0] hn / beta, [1] est, [2] |b|^2, [3] |r|^2, [4] |w|^2 before
  const double bnorm = dev_norm(h, K, b, sc + 2);
  fpc_info inf{};
  if (bnorm == 0.0) {
    FPC_HIP(hipMemsetAsync(x, 0, N * sizeof(double), s));
    FPC_HIP(hipStreamSynchronize(s));
    inf.converged = 1;
    inf.seconds = now_s() - t0;
    if (info) *info = inf;
    return FPC_OK;
  }
  if (!use_x0) FPC_HIP(hipMemsetAsync(x, 0, N * sizeof(double), s));
  const double tol = rtol * bnorm;
  const bool dcgs = h->opt.ortho == FPC_DCGS2 && dcgs_supported(N);
  int its = 0, cycles = 0;
  bool converged = false;
  double est = 1.0, truer = 1.0;
  while (true) {
    // true residual r = b - J x
    matvec(h, trans, x, K.w.p);
    FPC_HIP(hipMemcpyAsync(K.r.p, b, N * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    axpby(-1.0, K.w.p, 1.0, K.r.p, N, s);
    mdot(K.r.p, 0, 1, K.r.p, N, K.partials.p, sc + 3, s);
    gmres_init(K.g.p, m, sc + 3, sc, s);
    const double beta = std::sqrt(std::max(read_f64(sc + 3, s), 0.0));
    truer = beta / bnorm;
    if (beta <= tol) {
      converged = true;
      break;
    }
    if (its >= h->opt.maxit) break;
    scale_by_inv(K.r.p, sc, K.V.p, N, s);
    const int k = dcgs ? dcgs2_cycle(h, K, trans, tol, its, est)
                       : cgs_cycle(h, K, trans, tol, its, est);
    est /= bnorm;
    gmres_trisolve(K.H.p, m, K.g.p, K.y.p, k, s);
    // x += Z y  (maxpy subtracts, so negate y on the device)
    axpby(-1.0, K.y.p, 0.0, K.h1.p, k, s);
    maxpy(K.Z.p, N, k, K.h1.p, x, N, s);
    ++cycles;
  }
  inf.iterations = its;
  inf.restarts = cycles;
  inf.converged = converged ? 1 : 0;
  inf.true_rel_residual = truer;
  inf.est_rel_residual = est;
  inf.seconds = now_s() - t0;
  if (info) *info = inf;
  return converged ? FPC_OK : FPC_NOT_CONVERGED;
}

// ------------------------------------------------------------- batches
// Operators of the batched V-cycle: sliced ELL, or for rows of 32 blocks
// and more on average (the restrictions, coarse operators) the row-group
// layout read by one wavefront per row, by four from 256 blocks on (the
// restriction onto the coarsest level has a few hundred rows of about a
// thousand blocks).
template <typename T>
void batch_op(const Bsr& a, Op<T>& op, hipStream_t s) {
  if (a.nbr > 0 && a.nnzb >= 32 * a.nbr) {
    op.fmt = a.nnzb >= 256 * a.nbr ? 2 : 1;
    bsr_to_vrow(a, kBatchRowGroup, op.v, s);
  } else {
    op.fmt = 0;
    bsr_to_sell(a, op.s, s);
  }
}

void ensure_batch_ops(fpc_handle* h) {
  hipStream_t s = h->stream;
  const bool fp32 = h->opt.precision == FPC_FP32_PREC;
  for (Level& L : h->amg.L) {
    if (L.coarsest) continue;
    if (fp32 ? L.gA.rows() != 0 : L.bA.rows() != 0) continue;
    if (fp32) {
      batch_op(L.A, L.gA, s);
      batch_op(L.P, L.gP, s);
      batch_op(L.R, L.gR, s);
    } else {
      batch_op(L.A, L.bA, s);
      batch_op(L.P, L.bP, s);
      batch_op(L.R, L.bR, s);
    }
  }
  FPC_HIP(hipStreamSynchronize(s));
}

BatchWork& batch_work(fpc_handle* h, int KB) {
  BatchWork* w = &h->bw;
  const int m = h->opt.restart;
  if (w->KB == KB && w->m == m && w->N == h->N) return *w;
  w->KB = KB;
  w->m = m;
  w->N = h->N;
  const int64_t N = h->N;
  w->V.alloc((int64_t)(m + 1) * N * KB);
  w->Z.alloc((int64_t)m * N * KB);
  w->W.alloc(N * KB);
  w->R.alloc(N * KB);
  w->Bi.alloc(N * KB);
  w->Xi.alloc(N * KB);
  w->tt.alloc(std::max<int64_t>(h->n_t, 1) * KB);
  w->H.alloc((int64_t)KB * (m + 1) * m);
  w->cs.alloc((int64_t)KB * m);
  w->sn.alloc((int64_t)KB * m);
  w->g.alloc((int64_t)KB * (m + 1));
  w->y.alloc((int64_t)KB * m);
  w->yneg.alloc((int64_t)KB * m);
  w->h1.alloc((int64_t)KB * (m + 1));
  w->h2.alloc((int64_t)KB * (m + 1));
  w->nrm2.alloc(KB);
  w->beta2.alloc(KB);
  w->scal.alloc(KB);
  w->est.alloc(KB);
  w->bnorm2.alloc(KB);
  w->partials.alloc(bdot_partials(2 * (m + 1) + 1, KB));
  w->D.alloc((int64_t)(2 * (m + 1) + 1) * KB);
  w->P.alloc((int64_t)(m + 1) * KB);
  w->rho.alloc(KB);
  w->ww.alloc(KB);
  w->sc.alloc(3 * KB);
  w->active.alloc(KB);
  w->kc.alloc(KB);
  w->brk.alloc(KB);
  w->pf.alloc(KB);
  w->needfin.alloc(KB);
  psolve_batch_buffers(h->ps, KB);
  return *w;
}

void matvec_b(fpc_handle* h, const double* X, double* Y, int KB) {
  hipStream_t s = h->stream;
  const int64_t nu = h->n_u, nt = h->n_t;
  const double *Xu = X, *Xt = X + nu * KB, *Xp = X + (nu + nt) * KB;
  double *Yu = Y, *Yt = Y + nu * KB, *Yp = Y + (nu + nt) * KB;
  sell_mv_b(h->sAJ, Xu, Yu, KB, s);
  csr_spmv2_b(&h->C1, Xt, 1.0, &h->Q1, Xp, 1.0, Yu, 1.0, KB, s);
  csr_spmv2_b(&h->C2, Xu, 1.0, &h->H, Xt, -1.0, Yt, 0.0, KB, s);
  csr_spmv2_b(&h->Q2, Xu, 1.0, &h->T, Xp, 1.0, Yp, 0.0, KB, s);
}

// Alg 3.4 on KB right-hand sides at once.  With Q2 = 0 the two AMG calls of a
// column combine into one (the V-cycle is linear), so the cycle runs on KB
// interleaved columns w_u + C1 t_t - Q1 v_p.
template <typename T, int NV>
void apply_fwd_b(fpc_handle* h, BatchWork& w, const double* W, double* V) {
  hipStream_t s = h->stream;
  const int KB = NV;
  const int64_t nu = h->n_u, nt = h->n_t, np = h->n_p;
  const double *Wu = W, *Wt = W + nu * KB, *Wp = W + (nu + nt) * KB;
  double *Vu = V, *Vt = V + nu * KB, *Vp = V + (nu + nt) * KB;
  face_apply_b(h->hinv.p, Wt, w.tt.p, np, KB, 0, s);
  psolve_apply_b(h->ps, Wp, Vp, np, KB, s);
  CycleVecs<T>& cv = cycle_vecs<T>(h->amg, NV);
  to_level_b<T>(cv.lv[0].b.p, KB, nu, Wu, h->C1, w.tt.p, 1.0, h->Q1, Vp, -1.0,
                s);
  vcycle<T, NV>(h->amg, false, s);
  from_level_b<T>(cv.lv[0].xo.p, nu, KB, Vu, s);
  tface_b(h->C2, Vu, w.tt.p, h->hinv.p, Vt, np, KB, s);
}

void apply_b(fpc_handle* h, BatchWork& w, const double* W, double* V) {
  const bool fp32 = h->opt.precision == FPC_FP32_PREC;
  if (w.KB == 8) {
    if (fp32) apply_fwd_b<float, 8>(h, w, W, V);
    else apply_fwd_b<double, 8>(h, w, W, V);
  } else {
    if (fp32) apply_fwd_b<float, 32>(h, w, W, V);
    else apply_fwd_b<double, 32>(h, w, W, V);
  }
}

// Block of k right-hand sides: every column runs its own FGMRES(m) with its
// own tolerance; the columns advance together so that the preconditioner and
// the Jacobian are applied to all active columns in one pass.
fpc_status fgmres_batch(fpc_handle* h, int k, const double* B, int64_t ldb,
                        double* X, int64_t ldx, double rtol, fpc_info* infos) {
  const double t0 = now_s();
  hipStream_t s = h->stream;
  if (h->opt.mode != FPC_TUP)
    throw Error(FPC_ERR_UNSUPPORTED, "batched solve uses the t-u-p mode");
  if (h->has_q2)
    throw Error(FPC_ERR_UNSUPPORTED,
                "batched solve needs Q2 = 0 (its two AMG calls share one cycle)");
  if (k < 1 || k > kMaxBatch)
    throw Error(FPC_ERR_ARG, "batched solve: 1 to 32 right-hand sides");
  const int KB = k <= 8 ? 8 : kMaxBatch;
  ensure_batch_ops(h);
  BatchWork& w = batch_work(h, KB);
  const int m = h->opt.restart;
  const int64_t N = h->N;
  if (rtol <= 0) rtol = h->opt.rtol;
  fill_i32(h->flags.p, 0, FLAG_COUNT, s);
  for (int c = 0; c < k; ++c) check_finite(B + c * ldb, N, h->flags.p, s);
  check_flags(h, "right-hand sides");
  pack_cols(B, ldb, N, k, KB, w.Bi.p, s);
  bmdot(w.Bi.p, 0, 1, w.Bi.p, N, KB, w.partials.p, w.bnorm2.p, s);
  std::vector<double> bn(KB), hbuf(KB);
  std::vector<int> act(KB, 0), kc(KB, 0), brk(KB, 0), done(KB, 0),
      conv(KB, 0), its(KB, 0), cycles(KB, 0);
  std::vector<double> truer(KB, 0.0), estv(KB, 0.0), hs(3 * KB, 0.0);
  std::vector<int> pfh(KB, 1), nf(KB, 0);
  const bool dcgs = h->opt.ortho == FPC_DCGS2 && bdcgs_supported(N, KB);
  FPC_HIP(hipMemcpyAsync(bn.data(), w.bnorm2.p, KB * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  FPC_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < KB; ++c) {
    bn[c] = std::sqrt(std::max(bn[c], 0.0));
    if (c >= k || bn[c] == 0.0) {
      done[c] = 1;
      conv[c] = 1;
    }
  }
  FPC_HIP(hipMemsetAsync(w.Xi.p, 0, N * KB * sizeof(double), s));
  int total = 0;
  while (true) {
    matvec_b(h, w.Xi.p, w.W.p, KB);
    FPC_HIP(hipMemcpyAsync(w.R.p, w.Bi.p, N * KB * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    bsub(w.R.p, w.W.p, N * KB, s);  // W = R - W = B - J X
    bmdot(w.W.p, 0, 1, w.W.p, N, KB, w.partials.p, w.beta2.p, s);
    FPC_HIP(hipMemcpyAsync(hbuf.data(), w.beta2.p, KB * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    FPC_HIP(hipStreamSynchronize(s));
    bool any = false;
    for (int c = 0; c < KB; ++c) {
      act[c] = 0;
      kc[c] = 0;
      if (done[c]) continue;
      const double beta = std::sqrt(std::max(hbuf[c], 0.0));
      truer[c] = beta / bn[c];
      if (beta <= rtol * bn[c]) {
        done[c] = 1;
        conv[c] = 1;
        continue;
      }
      act[c] = 1;
      any = true;
    }
    if (!any || total >= h->opt.maxit) break;
    FPC_HIP(hipMemcpyAsync(w.active.p, act.data(), KB * sizeof(int),
                           hipMemcpyHostToDevice, s));
    bgmres_init(w.g.p, m, KB, w.beta2.p, w.active.p, w.scal.p, s);
    bscale(w.W.p, w.scal.p, w.V.p, N, KB, s);
    for (int c = 0; c < KB; ++c)
      if (act[c]) ++cycles[c];
    int jlast = 0;
    if (dcgs) {
      // delayed Gram-Schmidt per column, as dcgs2_cycle: the decision on the
      // provisional estimate, a finalizing pass for the columns that stop
      fill_i32(w.pf.p, 1, KB, s);
      std::fill(pfh.begin(), pfh.end(), 1);
      const int64_t stride = N * KB;
      auto fetch = [&]() {
        FPC_HIP(hipMemcpyAsync(hs.data(), w.sc.p, 3 * KB * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        FPC_HIP(hipStreamSynchronize(s));
      };
      for (int j = 0; j < m; ++j) {
        double* Uj = w.V.p + (int64_t)j * stride;
        double* Zj = w.Z.p + (int64_t)j * stride;
        apply_b(h, w, Uj, Zj);
        matvec_b(h, Zj, w.W.p, KB);
        bdcgs_dot(w.V.p, stride, j + 1, Uj, w.W.p, N, KB, w.partials.p, w.D.p,
                  s);
        bdcgs_finish(w.D.p, j + 1, true, nullptr, w.H.p, m, w.cs.p, w.sn.p,
                     w.g.p, w.P.p, w.rho.p, w.ww.p, w.sc.p, w.pf.p,
                     w.active.p, KB, s);
        bdcgs_update(w.V.p, stride, j, w.D.p, w.P.p, w.rho.p, w.W.p, N, KB,
                     w.partials.p, s);
        bdcgs_peek(w.partials.p, N, w.H.p, m, w.cs.p, w.sn.p, w.g.p, w.P.p, j,
                   w.ww.p, w.sc.p, w.pf.p, w.active.p, KB, s);
        fetch();
        ++total;
        jlast = j;
        bool changed = false, any_nf = false, any_last = false, others = false;
        auto stop = [&](int c, int kcol) {
          act[c] = 0;
          kc[c] = kcol;
          changed = true;
        };
        for (int c = 0; c < KB; ++c) {
          nf[c] = 0;
          if (!act[c]) continue;
          const double tol = rtol * bn[c];
          const int code = (int)hs[2 * KB + c];
          const bool was_fin = j > 0 && !pfh[c];  // column j - 1 made final now
          pfh[c] = 0;
          if (code == 2) {  // u_j inside the basis: column j - 1 is the last
            estv[c] = hs[KB + c];
            pfh[c] = 1;
            stop(c, j);
            continue;
          }
          if (was_fin && hs[KB + c] <= tol) {
            // column j - 1 meets the tolerance: the step only made it final
            estv[c] = hs[KB + c];
            stop(c, j);
            continue;
          }
          ++its[c];
          if (code == 1) {  // breakdown: column j committed as it is
            estv[c] = hs[KB + c];
            pfh[c] = 1;
            stop(c, j + 1);
            continue;
          }
          estv[c] = hs[c];
          const bool last = j + 1 == m || its[c] >= h->opt.maxit ||
                            total >= h->opt.maxit;
          if (hs[c] <= tol || last) {
            nf[c] = 1;
            any_nf = true;
            any_last = any_last || last;
          } else {
            others = true;
          }
        }
        // A column whose provisional estimate meets the tolerance while
        // others go on stays one more step, whose first pass makes its
        // column final at no extra cost (the block is processed whole); the
        // finalizing pass runs when no active column goes on, or at the end
        // of the cycle or of the iteration budget.
        if (any_nf && !any_last && others) any_nf = false;
        if (any_nf) {
          FPC_HIP(hipMemcpyAsync(w.needfin.p, nf.data(), KB * sizeof(int),
                                 hipMemcpyHostToDevice, s));
          bdcgs_dot(w.V.p, stride, j + 2, w.V.p + (int64_t)(j + 1) * stride,
                    nullptr, N, KB, w.partials.p, w.D.p, s);
          bdcgs_finish(w.D.p, j + 2, false, w.needfin.p, w.H.p, m, w.cs.p,
                       w.sn.p, w.g.p, w.P.p, w.rho.p, w.ww.p, w.sc.p, w.pf.p,
                       w.active.p, KB, s);
          fetch();
          for (int c = 0; c < KB; ++c) {
            if (!nf[c]) continue;
            pfh[c] = 1;
            estv[c] = hs[KB + c];
            const bool last = j + 1 == m || its[c] >= h->opt.maxit ||
                              total >= h->opt.maxit;
            if (hs[KB + c] <= rtol * bn[c] || last || (int)hs[2 * KB + c] == 2)
              stop(c, j + 1);
          }
        }
        bool still = false;
        for (int c = 0; c < KB; ++c) still = still || act[c];
        if (!still || total >= h->opt.maxit) break;
        if (changed)
          FPC_HIP(hipMemcpyAsync(w.active.p, act.data(), KB * sizeof(int),
                                 hipMemcpyHostToDevice, s));
      }
    } else {
      for (int j = 0; j < m; ++j) {
        const int64_t stride = N * KB;
        double* Vj = w.V.p + (int64_t)j * stride;
        double* Zj = w.Z.p + (int64_t)j * stride;
        apply_b(h, w, Vj, Zj);
        matvec_b(h, Zj, w.W.p, KB);
        // classical Gram-Schmidt twice in three passes, per column: h1 with
        // |w|^2 (in h1 row j + 1), w -= V h1 with h2, w -= V h2 with |w|^2
        bcgs_dot(w.V.p, stride, j + 1, w.W.p, N, KB, w.partials.p, w.h1.p, s);
        bcgs_axpy_dot(w.V.p, stride, j + 1, w.h1.p, w.W.p, N, KB, w.partials.p,
                      w.h2.p, s);
        bcgs_axpy_norm(w.V.p, stride, j + 1, w.h2.p, w.W.p, N, KB, w.partials.p,
                       w.nrm2.p, s);
        bgmres_step(w.H.p, w.cs.p, w.sn.p, w.g.p, w.h1.p, w.h2.p, w.nrm2.p,
                    w.h1.p + (int64_t)(j + 1) * KB, j, m, KB, w.active.p,
                    w.scal.p, w.est.p, w.brk.p, s);
        bscale(w.W.p, w.scal.p, w.V.p + (int64_t)(j + 1) * stride, N, KB, s);
        FPC_HIP(hipMemcpyAsync(estv.data(), w.est.p, KB * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        FPC_HIP(hipMemcpyAsync(brk.data(), w.brk.p, KB * sizeof(int),
                               hipMemcpyDeviceToHost, s));
        FPC_HIP(hipStreamSynchronize(s));
        ++total;
        jlast = j;
        bool changed = false, still = false;
        for (int c = 0; c < KB; ++c) {
          if (!act[c]) continue;
          ++its[c];
          if (estv[c] <= rtol * bn[c] || brk[c] || its[c] >= h->opt.maxit) {
            act[c] = 0;
            kc[c] = j + 1;
            changed = true;
          } else {
            still = true;
          }
        }
        if (!still || total >= h->opt.maxit) break;
        if (changed)
          FPC_HIP(hipMemcpyAsync(w.active.p, act.data(), KB * sizeof(int),
                                 hipMemcpyHostToDevice, s));
      }
    }
    for (int c = 0; c < KB; ++c)
      if (act[c]) kc[c] = jlast + 1;
    int kmax = 0;
    for (int c = 0; c < KB; ++c) kmax = std::max(kmax, kc[c]);
    FPC_HIP(hipMemcpyAsync(w.kc.p, kc.data(), KB * sizeof(int),
                           hipMemcpyHostToDevice, s));
    btrisolve(w.H.p, w.g.p, w.y.p, w.kc.p, m, KB, s);
    axpby(-1.0, w.y.p, 0.0, w.yneg.p, (int64_t)m * KB, s);
    bmaxpy(w.Z.p, N * KB, kmax, w.yneg.p, w.Xi.p, N, KB, s);
    for (int c = 0; c < KB; ++c)
      if (!done[c] && its[c] >= h->opt.maxit) done[c] = 1;
  }
  unpack_cols(w.Xi.p, N, k, KB, X, ldx, s);
  FPC_HIP(hipStreamSynchronize(s));
  const double secs = now_s() - t0;
  bool all = true;
  for (int c = 0; c < k; ++c) {
    all = all && conv[c];
    if (infos) {
      infos[c].iterations = its[c];
      infos[c].restarts = cycles[c];
      infos[c].converged = conv[c];
      infos[c].true_rel_residual = bn[c] > 0 ? truer[c] : 0.0;
      infos[c].est_rel_residual = bn[c] > 0 ? estv[c] / bn[c] : 0.0;
      infos[c].seconds = secs;
    }
  }
  return all ? FPC_OK : FPC_NOT_CONVERGED;
}

// Shapes and array presence of the seven blocks (nothing is read yet).
void check_block_shapes(const fpc_block_system* J) {
  const int64_t nu = J->n_u, nt = J->n_t, np = J->n_p;
  const struct { const fpc_csr* m; int64_t r, c; const char* name; } b[] = {
      {&J->A, nu, nu, "A"},  {&J->C1, nu, nt, "C1"}, {&J->Q1, nu, np, "Q1"},
      {&J->C2, nt, nu, "C2"}, {&J->H, nt, nt, "H"},  {&J->Q2, np, nu, "Q2"},
      {&J->T, np, np, "T"}};
  for (const auto& e : b) {
    if (e.m->nrows != e.r || e.m->ncols != e.c)
      throw Error(FPC_ERR_DIM, std::string(e.name) + ": shape mismatch");
    if (e.m->nnz < 0 || !e.m->rowptr ||
        (e.m->nnz > 0 && (!e.m->colind || !e.m->val)))
      throw Error(FPC_ERR_ARG, std::string(e.name) + ": null array");
  }
}

// The seven blocks from the caller into handle-owned device CSR, checked.
void upload_blocks(fpc_handle* h, const fpc_block_system* J) {
  hipStream_t s = h->stream;
  const int64_t nu = h->n_u, nt = h->n_t, np = h->n_p;
  upload_csr(J->A, J->ptr_space, nu, nu, h->A, s, "A");
  upload_csr(J->C1, J->ptr_space, nu, nt, h->C1, s, "C1");
  upload_csr(J->Q1, J->ptr_space, nu, np, h->Q1, s, "Q1");
  upload_csr(J->C2, J->ptr_space, nt, nu, h->C2, s, "C2");
  upload_csr(J->H, J->ptr_space, nt, nt, h->H, s, "H");
  upload_csr(J->Q2, J->ptr_space, np, nu, h->Q2, s, "Q2");
  upload_csr(J->T, J->ptr_space, np, np, h->T, s, "T");
  for (const Csr* m : {&h->A, &h->C1, &h->Q1, &h->C2, &h->H, &h->Q2, &h->T})
    csr_validate(*m, h->flags.p, s);
  // the coupling blocks of the u rows touch the fracture nodes only
  csr_active_rows(h->C1, s);
  csr_active_rows(h->Q1, s);
}

// Alg 3.3 cpt_tup / Alg 3.1 cpt_tpu on the uploaded blocks.  `prev`: the
// previous hierarchy, whose pattern-only parts are reused when the level-0
// block pattern is unchanged.
// update != 0: a numeric re-setup (fpc_update_values), which may keep the
// pattern-only parts of the previous construction; a setup builds everything.
void construct(fpc_handle* h, Hierarchy* prev, double t0, bool update) {
  hipStream_t s = h->stream;
  const int64_t nu = h->n_u, nt = h->n_t, np = h->n_p;
  h->has_q2 = h->Q2.nnz > 0;
  const double t1 = now_s();
  // H~ = Bdiag(H, 3) and its inverse
  h->hinv.alloc(std::max<int64_t>(np * 9, 1));
  hinv_setup(h->H, np, h->hinv.p, h->flags.p, s);
  check_flags(h, "H~ = Bdiag(H,3)");
  // S1 = A + C1 (H~^{-1} C2)
  Bsr C1b, Xb, CX, S1;
  h->Ab = Bsr();
  csr_to_bsr(h->A, 3, 3, h->Ab, s);
  csr_to_bsr(h->C1, 3, 3, C1b, s);
  csr_to_bsr(h->C2, 3, 3, Xb, s);
  bsr_block_row_scale(Xb, h->hinv.p, s);
  spgemm(C1b, Xb, CX, h->flags.p, s);
  bsr_add(h->Ab, CX, S1, s);
  check_flags(h, "S1 = A + C1 H~^-1 C2");
  if (h->has_q2 && h->opt.mode != FPC_TPU) {
    // Alg 3.3: [S_K]_k = Q2^(k)T S1^(k)^-1 Q1^(k)
    Csr Q1T;
    csr_transpose(h->Q1, Q1T, s);
    h->S_K.alloc(std::max<int64_t>(np, 1));
    fixed_stress(S1, Q1T, h->Q2, h->S_K.p, h->flags.p, s);
    check_flags(h, "fixed stress FS(Q2, S1, Q1)");
  } else if (h->has_q2) {
    // Alg 3.1: S~ = S1 - Q1 T~^-1 Q2, T~ = diag(T)
    Bsr Q1b, Q2b, QQ, St;
    csr_to_bsr(h->Q1, 3, 1, Q1b, s);
    csr_to_bsr(h->Q2, 1, 3, Q2b, s);
    bsr_row_scale_inv_diag(Q2b, h->T, -1.0, h->flags.p, s);
    spgemm(Q1b, Q2b, QQ, h->flags.p, s);
    bsr_add(S1, QQ, St, s);
    S1 = std::move(St);
    check_flags(h, "S~ = S1 - Q1 T~^-1 Q2");
  }
  bsr_to_sell(h->Ab, h->sAJ, s);
  // the previous hierarchy is reusable iff the operator it was built on has
  // the same block pattern (values and contact states may differ)
  if (prev) {
    const Bsr* A0 = prev->L.empty() ? nullptr : &prev->L[0].A;
    const bool same = A0 && A0->nbr == S1.nbr && A0->nnzb == S1.nnzb &&
                      same_pattern(A0->rowptr.p, A0->col.p, S1.rowptr.p,
                                   S1.col.p, S1.nbr, S1.nnzb, s);
    if (!same) prev = nullptr;
  }
  h->reused_hierarchy = prev != nullptr;
  const double t2 = now_s();
  build_psolve(h, update);
  const double t3 = now_s();
  build_hierarchy(h, std::move(S1), prev);
  const double t4 = now_s();
  h->t_t.alloc(std::max<int64_t>(nt, 1));
  h->tmp_p.alloc(std::max<int64_t>(np, 1));
  if (h->has_q2) {
    h->tmp_u.alloc(nu);
    h->tmp_p2.alloc(std::max<int64_t>(np, 1));
  }
  h->scratchN.alloc(h->N);
  // work vectors of the solve path, so that solves allocate nothing
  ensure_krylov(h, h->kry1, 1);
  if (h->opt.precision == FPC_FP32_PREC) cycle_vecs<float>(h->amg, 1);
  else cycle_vecs<double>(h->amg, 1);
  FPC_HIP(hipStreamSynchronize(s));
  h->ready = true;
  h->setup_times[0] = t4 - t0;
  h->setup_times[1] = t1 - t0;
  h->setup_times[2] = t2 - t1;
  h->setup_times[3] = t3 - t2;
  h->setup_times[4] = t4 - t3;
}

// Transmissibility gradient on a caller-chosen int32 work area of at least
// grad_scratch_words(n_p, n_pairs) words: pairs validated first, then the
// per-face lists and the sums.
void grad_run(fpc_handle* h, const fpc_flow_graph* g, const double* lam_p,
              const double* p, double* grad, int32_t* work) {
  hipStream_t s = h->stream;
  const int64_t m = g->n_pairs, n = g->n_p;
  fill_i32(h->flags.p, 0, FLAG_COUNT, s);
  grad_validate(n, m, g->pair_k, g->pair_l, work, h->flags.p, s);
  check_flags(h, "face pairs");
  grad_finish(n, m, g->pair_k, g->pair_l, g->ndir, g->upsilon, lam_p, p, grad,
              work, s);
  FPC_HIP(hipStreamSynchronize(s));
}

void grad_precheck(const fpc_handle* h, const fpc_flow_graph* g) {
  if (h->has_q2)
    throw Error(FPC_ERR_UNSUPPORTED,
                "transmissibility gradient assumes Q2 = 0 (Q2 depends on "
                "the transmissibility on open faces)");
  if (g->n_pairs > (INT32_MAX - 2 * g->n_p - 1) / 2)
    throw Error(FPC_ERR_ARG, "too many face pairs for int32 pair lists");
}

}  // namespace

// ------------------------------------------- allocation-free work area
// fpc_grad_log_trans_noalloc takes its work area from this file-scope device
// array instead of allocating one per call.  Every GPU holds its own copy
// until the process ends.  In host code the name `scratch` is only a host
// stand-in: the device address is looked up once per device
// (hipGetSymbolAddress, with that device current, in fpc_create) and kept in
// g_scratch_dev, which is what kernels receive.
constexpr int64_t kStaticScratchWords = int64_t(1) << 20;  // 4 MiB of int32
static __device__ __align__(256) int32_t scratch[kStaticScratchWords];

namespace {

constexpr int kMaxDevices = 64;
std::atomic<int> g_live_handles{0};  // handles created and not destroyed
std::mutex g_scratch_mu;
int32_t* g_scratch_dev[kMaxDevices] = {};

// Records the device address of `scratch` on `dev`, the current device.
void scratch_locate(int dev) {
  if (dev < 0 || dev >= kMaxDevices)
    throw Error(FPC_ERR_UNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev]) return;
  void* ptr = nullptr;
  FPC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) throw Error(FPC_ERR_HIP, "hipGetSymbolAddress returned NULL");
  g_scratch_dev[dev] = static_cast<int32_t*>(ptr);
}

int32_t* scratch_on(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  int32_t* ptr = (dev >= 0 && dev < kMaxDevices) ? g_scratch_dev[dev] : nullptr;
  if (!ptr) throw Error(FPC_ERR_STATE, "static work area not located");
  return ptr;
}

}  // namespace

// ================================================================= C ABI
extern "C" {

void fpc_default_options(fpc_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->mode = FPC_TUP;
  o->precision = FPC_FP64;
  o->restart = 50;
  o->maxit = 1000;
  o->rtol = 1e-8;
  o->max_batch = 32;
  o->graphs = 1;
  o->ortho = FPC_DCGS2;
  o->tune = 0;
  o->amg.max_coarse = 2000;
  o->amg.max_levels = 12;
  o->amg.cheb_degree = 2;
  o->amg.cheb_ratio = 5.0;
  o->amg.power_its = 10;
  o->amg.lam_safety = 1.1;
  o->amg.omega_factor = 4.0 / 3.0;
  o->amg.drop_tol = 1e-10;
}

fpc_status fpc_create(fpc_handle** hp, const fpc_options* opt, void* stream) {
  if (!hp) return FPC_ERR_ARG;
  *hp = nullptr;
  fpc_handle* h = nullptr;
  try {
    h = new fpc_handle();
  } catch (...) {
    return FPC_ERR_OOM;
  }
  if (opt) h->opt = *opt;
  else fpc_default_options(&h->opt);
  const fpc_options& o = h->opt;
  if ((o.mode != FPC_TUP && o.mode != FPC_TPU && o.mode != FPC_TUP_STAR) ||
      (o.precision != FPC_FP64 && o.precision != FPC_FP32_PREC) ||
      o.restart < 1 || o.restart + 1 > kMaxKrylov || o.maxit < 1 ||
      o.amg.cheb_degree != 2 || o.amg.max_levels < 1 || o.amg.power_its < 1 ||
      o.amg.cheb_ratio <= 1.0 || o.max_batch < 1 || o.max_batch > kMaxBatch ||
      (o.graphs != 0 && o.graphs != 1) || o.tune < 0 || o.tune > 2 ||
      (o.ortho != FPC_CGS2 && o.ortho != FPC_MGS && o.ortho != FPC_DCGS2)) {
    delete h;
    return FPC_ERR_ARG;
  }
  h->stream = (hipStream_t)stream;
  fpc_status st = guard(h, [&] {
    // keep freed device memory in the default pool of this device for reuse
    int dev = 0;
    FPC_HIP(hipGetDevice(&dev));
    h->device = dev;
    scratch_locate(dev);
    hipMemPool_t pool;
    FPC_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
    uint64_t keep = UINT64_MAX;
    FPC_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
    h->flags.alloc(FLAG_COUNT);
    FPC_HIP(hipMemsetAsync(h->flags.p, 0, FLAG_COUNT * sizeof(int), h->stream));
  });
  if (st != FPC_OK) {
    delete h;
    return st;
  }
  *hp = h;
  g_live_handles.fetch_add(1);
  return FPC_OK;
}

fpc_status fpc_setup(fpc_handle* h, const fpc_block_system* J) {
  if (!h || !J) return FPC_ERR_ARG;
  return guard(h, [&] {
    const double t0 = now_s();
    hipStream_t s = h->stream;
    h->ready = false;
    h->have_T = false;
    const int64_t nu = J->n_u, nt = J->n_t, np = J->n_p;
    if (nu <= 0 || nu % 3 || np < 0 || nt != 3 * np)
      throw Error(FPC_ERR_DIM, "need n_u = 3 * nodes and n_t = 3 * n_p");
    if (J->ptr_space != FPC_HOST && J->ptr_space != FPC_DEVICE)
      throw Error(FPC_ERR_ARG, "ptr_space");
    h->n_u = nu;
    h->n_t = nt;
    h->n_p = np;
    h->N = nu + nt + np;
    fill_i32(h->flags.p, 0, FLAG_COUNT, s);
    upload_blocks(h, J);
    h->has_coords = J->coords != nullptr;
    if (h->has_coords) {
      h->coords.alloc(nu);
      FPC_HIP(hipMemcpyAsync(h->coords.p, J->coords, nu * sizeof(double),
                             J->ptr_space == FPC_DEVICE ? hipMemcpyDeviceToDevice
                                                        : hipMemcpyHostToDevice,
                             s));
      check_finite(h->coords.p, nu, h->flags.p, s);
    }
    check_flags(h, "input");
    construct(h, nullptr, t0, false);
  });
}

#define FPC_REQUIRE_READY(h)                                  \
  do {                                                        \
    if (!(h)) return FPC_ERR_ARG;                             \
    if (!(h)->ready) {                                        \
      (h)->last_error = "call before a successful fpc_setup"; \
      return FPC_ERR_STATE;                                   \
    }                                                         \
  } while (0)

fpc_status fpc_update_values(fpc_handle* h, const fpc_block_system* J) {
  FPC_REQUIRE_READY(h);
  if (!J) return FPC_ERR_ARG;
  return guard(h, [&] {
    const double t0 = now_s();
    if (J->n_u != h->n_u || J->n_t != h->n_t || J->n_p != h->n_p)
      throw Error(FPC_ERR_DIM, "fpc_update_values: sizes differ from the setup");
    if (J->ptr_space != FPC_HOST && J->ptr_space != FPC_DEVICE)
      throw Error(FPC_ERR_ARG, "ptr_space");
    check_block_shapes(J);
    h->ready = false;
    h->have_T = false;
    fill_i32(h->flags.p, 0, FLAG_COUNT, h->stream);
    upload_blocks(h, J);
    check_flags(h, "input");
    Hierarchy prev = std::move(h->amg);
    h->amg = Hierarchy();
    construct(h, &prev, t0, true);
  });
}

fpc_status fpc_apply_prec(fpc_handle* h, const double* w, double* v) {
  FPC_REQUIRE_READY(h);
  if (!w || !v) return FPC_ERR_ARG;
  return guard(h, [&] { apply(h, 0, w, v); });
}

fpc_status fpc_apply_prec_T(fpc_handle* h, const double* w, double* v) {
  FPC_REQUIRE_READY(h);
  if (!w || !v) return FPC_ERR_ARG;
  return guard(h, [&] { apply(h, 1, w, v); });
}

fpc_status fpc_matvec(fpc_handle* h, int trans, const double* x, double* y) {
  FPC_REQUIRE_READY(h);
  if (!x || !y) return FPC_ERR_ARG;
  return guard(h, [&] { matvec(h, trans ? 1 : 0, x, y); });
}

fpc_status fpc_vcycle(fpc_handle* h, const double* b, double* x) {
  FPC_REQUIRE_READY(h);
  if (!b || !x) return FPC_ERR_ARG;
  return guard(h, [&] {
    hipStream_t s = h->stream;
    if (h->opt.precision == FPC_FP32_PREC) {
      CycleVecs<float>& cv = cycle_vecs<float>(h->amg, 1);
      to_level<float>(cv.lv[0].b.p, 1, 0, h->n_u, b, nullptr, nullptr, 0.0,
                      nullptr, nullptr, 0.0, s);
      vcycle<float, 1>(h->amg, false, s);
      from_level<float>(cv.lv[0].xo.p, 1, h->n_u, x, 0, s);
    } else {
      CycleVecs<double>& cv = cycle_vecs<double>(h->amg, 1);
      FPC_HIP(hipMemcpyAsync(cv.lv[0].b.p, b, h->n_u * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
      vcycle<double, 1>(h->amg, false, s);
      FPC_HIP(hipMemcpyAsync(x, cv.lv[0].xo.p, h->n_u * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    }
  });
}

fpc_status fpc_solve(fpc_handle* h, const double* b, double* x, double rtol,
                     int use_x0, fpc_info* info) {
  FPC_REQUIRE_READY(h);
  if (!b || !x) return FPC_ERR_ARG;
  fpc_status st = FPC_OK;
  fpc_status g = guard(h, [&] { st = fgmres(h, 0, b, x, rtol, use_x0, info); });
  return g != FPC_OK ? g : st;
}

fpc_status fpc_solve_T(fpc_handle* h, const double* gv, double* lam,
                       double rtol, fpc_info* info) {
  FPC_REQUIRE_READY(h);
  if (!gv || !lam) return FPC_ERR_ARG;
  fpc_status st = FPC_OK;
  fpc_status g = guard(h, [&] { st = fgmres(h, 1, gv, lam, rtol, 0, info); });
  return g != FPC_OK ? g : st;
}

fpc_status fpc_solve_batch(fpc_handle* h, int k, const double* B, int64_t ldb,
                           double* X, int64_t ldx, double rtol,
                           fpc_info* infos) {
  FPC_REQUIRE_READY(h);
  if (!B || !X || k < 1 || k > h->opt.max_batch || ldb < h->N || ldx < h->N)
    return FPC_ERR_ARG;
  fpc_status st = FPC_OK;
  fpc_status g = guard(h, [&] {
    st = fgmres_batch(h, k, B, ldb, X, ldx, rtol, infos);
  });
  return g != FPC_OK ? g : st;
}

fpc_status fpc_grad_log_trans(fpc_handle* h, const fpc_flow_graph* g,
                              const double* lam_p, const double* p,
                              double* grad) {
  FPC_REQUIRE_READY(h);
  if (!g || !lam_p || !p || !grad || g->n_p != h->n_p || g->n_pairs < 0 ||
      (g->n_pairs > 0 && (!g->pair_k || !g->pair_l)) ||
      (g->n_p > 0 && (!g->ndir || !g->upsilon)))
    return FPC_ERR_ARG;
  return guard(h, [&] {
    grad_precheck(h, g);
    DevBuf<int32_t> work(grad_scratch_words(g->n_p, g->n_pairs));
    grad_run(h, g, lam_p, p, grad, work.p);
  });
}

fpc_status fpc_grad_log_trans_noalloc(fpc_handle* h, const fpc_flow_graph* g,
                                      const double* lam_p, const double* p,
                                      double* grad) {
  FPC_REQUIRE_READY(h);
  if (!g || !lam_p || !p || !grad || g->n_p != h->n_p || g->n_pairs < 0 ||
      (g->n_pairs > 0 && (!g->pair_k || !g->pair_l)) ||
      (g->n_p > 0 && (!g->ndir || !g->upsilon)))
    return FPC_ERR_ARG;
  return guard(h, [&] {
    grad_precheck(h, g);
    const int64_t words = grad_scratch_words(g->n_p, g->n_pairs);
    if (words > kStaticScratchWords)
      throw Error(FPC_ERR_ARG,
                  "work area of 2 n_p + 1 + 2 n_pairs = " +
                      std::to_string(words) +
                      " int32 exceeds the static maximum of " +
                      std::to_string(kStaticScratchWords));
    grad_run(h, g, lam_p, p, grad, scratch_on(h->device));
  });
}

fpc_status fpc_psolve(fpc_handle* h, int trans, const double* w, double* v) {
  FPC_REQUIRE_READY(h);
  if (!w || !v || trans < 0 || trans > 1) return FPC_ERR_ARG;
  return guard(h, [&] { psolve_apply(h->ps, w, v, h->n_p, trans, h->stream); });
}

fpc_status fpc_stream_triad(fpc_handle* h, int64_t n, const double* b,
                            const double* c, double scalar, double* a) {
  if (!h || n < 0 || (n && (!a || !b || !c))) return FPC_ERR_ARG;
  return guard(h, [&] { stream_triad(b, c, scalar, a, n, h->stream); });
}

int fpc_hierarchy_reused(const fpc_handle* h) {
  return h ? (h->reused_hierarchy ? 1 : 0) : -1;
}

fpc_status fpc_dense_inverse(fpc_handle* h, int64_t n, double* D) {
  if (!h || n < 0 || (n > 0 && !D)) return FPC_ERR_ARG;
  if (n > 16384) return FPC_ERR_ARG;
  if (n == 0) return FPC_OK;
  return guard(h, [&] {
    hipStream_t s = h->stream;
    const int64_t npad = round64(n);
    DevBuf<double> P(npad * npad);
    dense_pad(D, n, npad, P.p, s);
    fill_i32(h->flags.p, 0, FLAG_COUNT, s);
    gj_inverse(P.p, npad, h->flags.p, s);
    check_flags(h, "dense inverse");
    FPC_HIP(hipMemcpy2DAsync(D, n * sizeof(double), P.p, npad * sizeof(double),
                             n * sizeof(double), n, hipMemcpyDeviceToDevice,
                             s));
    FPC_HIP(hipStreamSynchronize(s));
  });
}

fpc_status fpc_pressure_info(const fpc_handle* h, fpc_pressure_desc* d) {
  if (!h || !d) return FPC_ERR_ARG;
  if (!h->ready) return FPC_ERR_STATE;
  *d = fpc_pressure_desc{};
  const PSolve& ps = h->ps;
  d->n_levels = ps.n_levels;
  d->n_fronts = ps.n_fronts;
  d->factor_entries = psolve_factor_entries(ps);
  d->solve_bytes = psolve_solve_bytes(ps);
  for (int64_t f = 0; f < ps.n_fronts; ++f) {
    d->max_pivots = std::max<int64_t>(d->max_pivots, ps.hm[f]);
    d->max_boundary = std::max<int64_t>(d->max_boundary, ps.hk[f]);
  }
  return FPC_OK;
}

int fpc_num_levels(const fpc_handle* h) {
  return (h && h->ready) ? (int)h->amg.L.size() : 0;
}

fpc_status fpc_level_info(const fpc_handle* h, int level, fpc_level_desc* d) {
  if (!h || !d) return FPC_ERR_ARG;
  if (!h->ready) return FPC_ERR_STATE;
  if (level < 0 || level >= (int)h->amg.L.size()) return FPC_ERR_ARG;
  const Level& L = h->amg.L[level];
  if (L.nnz_scalar < 0) {
    // counted on the first query (reporting only, not needed by the setup)
    fpc_handle* hh = const_cast<fpc_handle*>(h);
    const fpc_status st = guard(hh, [&] {
      hh->amg.L[level].nnz_scalar = bsr_count_nonzeros(L.A, h->stream);
    });
    if (st != FPC_OK) return st;
  }
  d->n_nodes = L.n_nodes;
  d->n_dofs = L.n_dofs_real;
  d->block = L.bs;
  d->nnzb = L.A.nnzb;
  d->nnz_scalar = L.nnz_scalar;
  d->p_nnzb = L.coarsest ? 0 : L.P.nnzb;
  d->r_nnzb = L.coarsest ? 0 : L.R.nnzb;
  d->lam_hi = L.lam_hi;
  d->n_agg = L.coarsest ? 0 : L.n_agg;
  for (int k = 0; k < 3; ++k) {
    d->layout[k] = L.coarsest ? 0 : L.layout[k];
    d->tune_us[k] = L.coarsest ? 0.0 : L.tune_us[k];
  }
  return FPC_OK;
}

fpc_status fpc_export_aggregates(const fpc_handle* h, int level, int32_t* agg,
                                 int32_t* rank) {
  if (!h) return FPC_ERR_ARG;
  if (!h->ready) return FPC_ERR_STATE;
  if (level < 0 || level >= (int)h->amg.L.size()) return FPC_ERR_ARG;
  const Level& L = h->amg.L[level];
  if (L.coarsest) return FPC_ERR_ARG;
  fpc_handle* hh = const_cast<fpc_handle*>(h);
  return guard(hh, [&] {
    if (agg)
      FPC_HIP(hipMemcpyAsync(agg, L.agg.p, L.n_nodes * sizeof(int32_t),
                             hipMemcpyDeviceToHost, h->stream));
    if (rank)
      FPC_HIP(hipMemcpyAsync(rank, L.rank.p, L.n_agg * sizeof(int32_t),
                             hipMemcpyDeviceToHost, h->stream));
    FPC_HIP(hipStreamSynchronize(h->stream));
  });
}

fpc_status fpc_export_level_matrix(const fpc_handle* h, int level, int which,
                                   int64_t* rowptr, int32_t* col, double* val) {
  if (!h || !rowptr || !col || !val) return FPC_ERR_ARG;
  if (!h->ready) return FPC_ERR_STATE;
  if (level < 0 || level >= (int)h->amg.L.size()) return FPC_ERR_ARG;
  const Level& L = h->amg.L[level];
  const Bsr* M = which == 0 ? &L.A : which == 1 ? &L.P : which == 2 ? &L.R : nullptr;
  if (!M || (which != 0 && L.coarsest)) return FPC_ERR_ARG;
  fpc_handle* hh = const_cast<fpc_handle*>(h);
  return guard(hh, [&] {
    FPC_HIP(hipMemcpyAsync(rowptr, M->rowptr.p, (M->nbr + 1) * sizeof(int64_t),
                           hipMemcpyDeviceToHost, h->stream));
    if (M->nnzb) {
      FPC_HIP(hipMemcpyAsync(col, M->col.p, M->nnzb * sizeof(int32_t),
                             hipMemcpyDeviceToHost, h->stream));
      FPC_HIP(hipMemcpyAsync(val, M->val.p,
                             M->nnzb * M->br * M->bc * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
    }
    FPC_HIP(hipStreamSynchronize(h->stream));
  });
}

fpc_status fpc_setup_times(const fpc_handle* h, double* t5) {
  if (!h || !t5) return FPC_ERR_ARG;
  for (int i = 0; i < 5; ++i) t5[i] = h->setup_times[i];
  return FPC_OK;
}

fpc_status fpc_kernel_timer(fpc_handle* h, int enable, int reset,
                            int64_t* launches, double* total_ms) {
  if (!h) return FPC_ERR_ARG;
  return guard(h, [&] {
    KTimer& t = h->ktimer;
    t.flush();
    if (launches) *launches = t.launches;
    if (total_ms) *total_ms = t.total_ms;
    if (reset) {
      t.launches = 0;
      t.total_ms = 0.0;
    }
    t.on = enable != 0;
    h->amg.timer = t.on ? &t : nullptr;
  });
}

fpc_status fpc_hash32_device(fpc_handle* h, uint32_t first, int64_t n,
                             uint32_t* out) {
  if (!h || !out || n < 0) return FPC_ERR_ARG;
  return guard(h, [&] {
    hash32_range(first, n, out, h->stream);
    FPC_HIP(hipStreamSynchronize(h->stream));
  });
}

void fpc_destroy(fpc_handle* h) {
  if (!h) return;
  // finish the handle's work, release (buffers go to the block cache on
  // their stream; the last handle returns the cache to the pool), then wait
  // for the releases
  hipStream_t s = h->stream;
  if (s) (void)hipStreamSynchronize(s);
  else (void)hipDeviceSynchronize();
  delete h;
  if (g_live_handles.fetch_sub(1) == 1) dev_cache_trim();
  if (s) (void)hipStreamSynchronize(s);
  else (void)hipDeviceSynchronize();
}

const char* fpc_status_string(fpc_status s) {
  switch (s) {
    case FPC_OK: return "ok";
    case FPC_NOT_CONVERGED: return "not converged";
    case FPC_ERR_ARG: return "invalid argument";
    case FPC_ERR_DIM: return "inconsistent dimensions";
    case FPC_ERR_PATTERN: return "invalid sparsity pattern";
    case FPC_ERR_SINGULAR_BLOCK: return "singular block";
    case FPC_ERR_NOT_SPD: return "pressure block not positive definite";
    case FPC_ERR_NAN: return "non-finite value";
    case FPC_ERR_HIP: return "HIP runtime error";
    case FPC_ERR_OOM: return "out of device memory";
    case FPC_ERR_STATE: return "handle not set up";
    case FPC_ERR_UNSUPPORTED: return "unsupported case";
  }
  return "unknown status";
}

const char* fpc_last_error(const fpc_handle* h) {
  return h ? h->last_error.c_str() : "null handle";
}

}  // extern "C"
