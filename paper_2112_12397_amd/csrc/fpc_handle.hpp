// Handle, hierarchy and work-vector structures of the fracprec library.
#pragma once

#include <array>
#include <string>
#include <vector>

#include "fpc_internal.hpp"

namespace fpc {

// One level of the smoothed-aggregation hierarchy.  Block rows are "nodes":
// mesh nodes (3 dofs) on level 0, aggregates (nb dofs, padded) below.
struct Level {
  int bs = 3;               // dofs per node on this level
  int nb = 6;               // dofs per node on the next level
  int64_t n_nodes = 0;
  int64_t n_dofs_real = 0;  // without padding dofs
  Bsr A, P, R;              // FP64 block CSR (setup, export, transposes)
  Bsr Pt;                   // tentative prolongator (kept for re-setups)
  // patterns of A P_tent, A P and R (A P) (kept for re-setups: the numeric
  // phase of each product runs on them)
  BsrPattern pat_ap0, pat_ap, pat_ac;
  TransposePlan plan_r;     // R = P^T
  Sell<double> sA;          // FP64 A in sliced ELL (power iteration)
  Op<double> oA, oP, oR;    // apply operators (layouts: rule or timing)
  Op<float> fA, fP, fR;
  Bsr AT;                   // A^T for the transposed cycle (lazy)
  Op<double> oAT;
  Op<float> fAT;
  int layout[3] = {0, 0, 0};   // layout of A, P, R (1 = sliced ELL, else lanes)
  double tune_us[3] = {0, 0, 0};  // timed winner per product (us), 0 by rule
  // multi-right-hand-side operators (sliced ELL, one thread per row and
  // column), built on the first batched solve
  Op<double> bA, bP, bR;
  Op<float> gA, gP, gR;
  DevBuf<double> dinv;      // n_nodes * bs
  DevBuf<float> dinv32;
  DevBuf<int32_t> agg;      // aggregate of every node (-1 isolated)
  DevBuf<int32_t> rank;     // kept modes per aggregate (n_agg)
  DevBuf<int32_t> node_rank;// real dofs per node (coarse levels)
  int64_t n_agg = 0;
  int64_t nnz_scalar = -1;  // nonzero scalars of A (counted when queried)
  double lam_hi = 0, theta = 0, delta = 0, c1 = 0, c2 = 0;
  bool coarsest = false;
};

template <typename T>
struct LevelVecs {
  DevBuf<T> x, xo, d, r, res, b;
  DevBuf<T> d0;  // first Chebyshev direction D^{-1} b / theta
};

// Per (precision, column count) set of level vectors.
template <typename T>
struct CycleVecs {
  int nv = 0;
  std::vector<LevelVecs<T>> lv;
};

// HIP-event timer around one kernel of the V-cycle (the level-0 residual
// SpMV), used for reporting its achieved bandwidth.
struct KTimer {
  bool on = false;
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  int64_t launches = 0;
  double total_ms = 0.0;
  void begin(hipStream_t s) {
    if (!on) return;
    if (ev.empty()) {
      ev.resize(4096);
      for (auto& e : ev) FPC_HIP(hipEventCreate(&e));
    }
    if (used + 2 > ev.size()) flush();
    FPC_HIP(hipEventRecord(ev[used], s));
  }
  void end(hipStream_t s) {
    if (!on) return;
    FPC_HIP(hipEventRecord(ev[used + 1], s));
    used += 2;
  }
  void flush() {
    if (used == 0) return;
    FPC_HIP(hipEventSynchronize(ev[used - 1]));
    for (size_t i = 0; i < used; i += 2) {
      float ms = 0.f;
      FPC_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
      total_ms += ms;
      ++launches;
    }
    used = 0;
  }
  ~KTimer() {
    for (auto& e : ev) (void)hipEventDestroy(e);
  }
};

// Captured V-cycles, keyed by (precision, column count).  The graphs refer to
// the level operators and vectors of one hierarchy and are dropped with it.
struct GraphCache {
  struct Slot {
    int key;
    hipGraph_t g;
    hipGraphExec_t e;
  };
  std::vector<Slot> slots;
  hipStream_t cap = nullptr;  // private stream used only for capturing
  GraphCache() = default;
  GraphCache(const GraphCache&) = delete;
  GraphCache& operator=(const GraphCache&) = delete;
  ~GraphCache() {
    clear();
    if (cap) (void)hipStreamDestroy(cap);
  }
  void clear() {
    for (Slot& s : slots) {
      if (s.e) (void)hipGraphExecDestroy(s.e);
      if (s.g) (void)hipGraphDestroy(s.g);
    }
    slots.clear();
  }
  hipGraphExec_t find(int key) const {
    for (const Slot& s : slots)
      if (s.key == key) return s.e;
    return nullptr;
  }
};

struct Hierarchy {
  KTimer* timer = nullptr;
  GraphCache* graphs = nullptr;  // non-null: batched V-cycles replay graphs
  std::vector<Level> L;
  int64_t nc = 0, ncpad = 0;  // coarsest dofs (padded) and dense size
  DevBuf<double> Ainv;        // ncpad x ncpad, row-major
  DevBuf<double> AinvT;       // transpose (lazy)
  std::vector<CycleVecs<double>> v64;
  std::vector<CycleVecs<float>> v32;
  bool have_transpose = false;
};

// Exact pressure-block solve: nested-dissection multifrontal factorization
// of S~2 (T when Q2 is empty).  Fronts are numbered level by level (leaves
// first); front f eliminates positions [f_slo, f_slo + f_m) of the order and
// couples to the f_k boundary positions bnd[f_bnd[f] ..]; its dense matrix
// (ld = m + k, row-major) starts at F + f_F[f], rows 0..m-1 holding
// [F11^-1 | F11^-1 F12] after the factorization.
struct PSolve {
  int64_t n = 0;
  int n_levels = 0;
  int64_t n_fronts = 0, n_slots = 0, F_words = 0;
  bool spd = true;
  std::vector<int64_t> lev_off;          // fronts of level l
  std::vector<int32_t> hm, hk;           // host copies of f_m, f_k
  DevBuf<int32_t> perm, pos;             // order: perm[position] = face
  DevBuf<int32_t> f_slo, f_m, f_k;
  DevBuf<int64_t> f_bnd, f_F;
  DevBuf<int32_t> bnd;                   // boundary positions, ascending
  DevBuf<int64_t> ch_off;                // children of f: ch[ch_off[f+1] ..
  DevBuf<int32_t> ch;                    //   ch_off[f+2])
  DevBuf<int64_t> g_off;                 // per position: contribution slots
  DevBuf<int32_t> g_slot;                //   (f_bnd[f] + a) to subtract
  DevBuf<double> F;
  // solve work lists per level: (front, first output) forward,
  // (front, first row) backward
  std::vector<int64_t> fwd_off, bwd_off;
  DevBuf<int2> fwd_items, bwd_items;
  DevBuf<double> xp, contrib;            // single column
  int KB = 0;                            // batch columns of the buffers below
  DevBuf<double> bpB, xpB, contribB;
  // numeric phase per level: fronts inverted in LDS (small), larger fronts
  // (big, host list), 64 x 64 tiles (front, ti, tj) of W and of the Schur
  // complements; host offsets of the front matrices
  std::vector<int64_t> small_off, w_off, s_off, hF;
  std::vector<std::vector<int32_t>> big;
  DevBuf<int32_t> small;
  DevBuf<int4> w_items, s_items;
  // the matrix the factor was computed from, for reuse on unchanged input
  DevBuf<int64_t> in_rp;
  DevBuf<int32_t> in_col;
  DevBuf<double> in_val, in_sk;
  bool has_sk = false;
};

// Per right-hand-side block of Krylov work space.
struct Krylov {
  int m = 0, k = 0;
  int64_t N = 0;
  DevBuf<double> V, Z;        // (m+1) x N x k, m x N x k
  DevBuf<double> w, r, tmp;   // N x k
  DevBuf<double> H, cs, sn, g, y;  // small arrays (device)
  DevBuf<double> h1, h2, scal, partials;
  DevBuf<double> D, P;        // delayed Gram-Schmidt: dot outputs, column
  DevBuf<int> ctrl;
  double* host = nullptr;     // pinned mirror for scalars read each step
  hipEvent_t ev = nullptr;    // marks the arrival of those scalars
  ~Krylov() {
    if (ev) (void)hipEventDestroy(ev);
    if (host) (void)hipHostFree(host);
  }
};

// Work space of the batched solve (KB interleaved right-hand sides).
struct BatchWork {
  int KB = 0, m = 0;
  int64_t N = 0;
  DevBuf<double> V, Z, W, R, Bi, Xi, tt;
  DevBuf<double> H, cs, sn, g, y, yneg, h1, h2, nrm2, beta2, scal, est,
      bnorm2, partials;
  DevBuf<double> D, P, rho, ww, sc;  // delayed Gram-Schmidt
  DevBuf<int> active, kc, brk, pf, needfin;
};

}  // namespace fpc

struct fpc_handle {
  fpc_options opt{};
  hipStream_t stream = nullptr;
  int device = 0;              // current device at fpc_create
  bool ready = false;
  int64_t n_u = 0, n_t = 0, n_p = 0, N = 0;
  fpc::Csr A, C1, Q1, C2, H, Q2, T;
  fpc::Csr C1T, C2T, Q1T, Q2T, HT, TT;
  bool have_T = false;
  fpc::Bsr Ab;                 // A as 3x3 blocks (J matvec)
  fpc::Sell<double> sAJ, sAJT;
  fpc::DevBuf<double> hinv;    // n_p * 9
  fpc::DevBuf<double> coords;  // n_nodes * 3 (optional)
  bool has_coords = false;
  fpc::Hierarchy amg;
  fpc::PSolve ps;
  fpc::DevBuf<int> flags;
  // apply-path scratch (FP64)
  fpc::DevBuf<double> t_t, tmp_u, tmp_u2, tmp_p, tmp_p2, scratchN;
  bool has_q2 = false;          // open faces: Q2 not empty
  bool reused_hierarchy = false;  // last construction reused the AMG patterns
  fpc::DevBuf<double> S_K;     // fixed-stress diagonal (t-u-p with Q2)
  fpc::Krylov kry1;            // single right-hand side
  fpc::Krylov kryB;            // batched
  fpc::KTimer ktimer;
  fpc::GraphCache graphs;
  fpc::BatchWork bw;
  std::string last_error;
  double setup_times[5] = {0, 0, 0, 0, 0};
};
