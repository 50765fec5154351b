"""Smoothed-aggregation AMG used as the inner ``AMG(K, y)`` operator.

The paper applies the Schur-complement inverse with an aggregation-based
multigrid (Sec. 3.1, PETSc GAMG) and gives no parameters.  This oracle
specifies one from published methods:

* strength: structure only (the node graph of the 3x3 block pattern),
* aggregation: distance-2 maximal independent set by synchronous max-rounds
  (Bell, Dalton & Olson, SIAM J. Sci. Comput. 34 (2012)), priorities from a
  fixed integer hash; aggregates = root + distance-1 neighbours, the rest
  joins a neighbouring aggregate,
* tentative prolongator: per-aggregate thin QR (modified Gram-Schmidt,
  applied twice) of the rigid-body near-nullspace, dependent columns dropped
  (Vanek, Mandel & Brezina, Computing 56 (1996)),
* smoothed prolongator ``P = (I - 4/3 / lambda_hi D^{-1} A) P_tent``,
  Galerkin coarse operator ``P^T A P``,
* Chebyshev smoothing of degree 2 on ``D^{-1} A`` over
  ``[lambda_hi / 5, lambda_hi]`` (Saad, Iterative Methods, Alg. 12.1; Adams
  et al., J. Comput. Phys. 188 (2003)), ``lambda_hi`` from 10 power
  iterations times 1.1.  The ratio 5 leaves the lowest fifth of the spectrum
  to the coarse space; with ratio 10 the degree-2 polynomial damps the upper
  part only by 1/2 and the iteration counts grow with the mesh,
* dense LU with partial pivoting on the coarsest level (<= 2000 dofs).
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .blocks import bool_product
from .hashing import hash32, hash_unit

IDX_BITS = 28
IDX_MASK = (1 << IDX_BITS) - 1


@dataclass
class AMGOptions:
    max_coarse: int = 2000
    max_levels: int = 12
    cheb_degree: int = 2
    cheb_ratio: float = 5.0
    power_its: int = 10
    lam_safety: float = 1.1
    omega_factor: float = 4.0 / 3.0
    drop_tol: float = 1e-10


@dataclass
class Level:
    A: sp.csr_matrix
    pattern: sp.csr_matrix          # node-level structural pattern
    node_ptr: np.ndarray            # dof range of each node
    key_stride: int                 # hash key of dof (node a, comp c) = stride*a + c
    B: np.ndarray                   # near-nullspace rows of this level
    dinv: np.ndarray = None
    AT: sp.csr_matrix = None
    lam_hi: float = 0.0
    theta: float = 0.0
    delta: float = 0.0
    P: sp.csr_matrix = None
    R: sp.csr_matrix = None
    P_tent: sp.csr_matrix = None
    agg: np.ndarray = None
    n_agg: int = 0
    rank: np.ndarray = None         # kept columns per aggregate

    @property
    def n_nodes(self):
        return self.node_ptr.size - 1

    @property
    def n(self):
        return self.A.shape[0]


def rigid_modes(coords, n_dofs):
    """Near-nullspace of 3D elasticity at the nodes: 3 translations and 3
    rotations about the centre of the bounding box (exact min/max, so the
    centre is reproducible bit for bit).  Without coordinates: translations.
    """
    nn = n_dofs // 3
    if coords is None:
        B = np.zeros((n_dofs, 3))
        for c in range(3):
            B[c::3, c] = 1.0
        return B
    X = np.asarray(coords, np.float64).reshape(nn, 3)
    ctr = 0.5 * (X.min(axis=0) + X.max(axis=0))
    y = X - ctr
    B = np.zeros((n_dofs, 6))
    for c in range(3):
        B[c::3, c] = 1.0
    # rotations about x, y, z: e_k x y
    B[1::3, 3], B[2::3, 3] = -y[:, 2], y[:, 1]
    B[0::3, 4], B[2::3, 4] = y[:, 2], -y[:, 0]
    B[0::3, 5], B[1::3, 5] = -y[:, 1], y[:, 0]
    return B


def _with_diag(G):
    n = G.shape[0]
    G = sp.csr_matrix(G.astype(np.int64) + sp.identity(n, dtype=np.int64,
                                                       format="csr"))
    G.data[:] = 1
    G.sort_indices()
    return G


def _max_nbr(G, vals):
    """max over the closed neighbourhood of every node (G holds the diagonal)."""
    return np.maximum.reduceat(vals[G.indices], G.indptr[:-1])


def mis2_aggregate(pattern, return_roots=False):
    """Distance-2 MIS aggregation on the structural node graph.

    Returns ``(agg, n_agg)``; ``agg[i] = -1`` marks isolated nodes (no
    off-diagonal block, e.g. Dirichlet nodes), which are not aggregated.
    With ``return_roots`` also the root node of every aggregate.

    Priority of node i: ``(hash32(i) << 28) | i`` (unique).  State 0 = out,
    1 = undecided, 2 = in; key = (state << 61) | priority.  Each synchronous
    round takes the maximum key over the closed distance-2 neighbourhood:
    an undecided node that is its own maximum joins the set, one whose
    maximum is an in-node leaves it.
    """
    G = _with_diag(pattern)
    n = G.shape[0]
    if n >= (1 << IDX_BITS):
        raise ValueError("too many nodes for the priority encoding")
    deg = np.diff(G.indptr)
    isolated = deg <= 1
    idx = np.arange(n, dtype=np.int64)
    prio = (hash32(idx).astype(np.int64) << IDX_BITS) | idx
    state = np.where(isolated, 0, 1).astype(np.int64)
    while True:
        und = state == 1
        if not und.any():
            break
        key = (state << 61) | prio
        m2 = _max_nbr(G, _max_nbr(G, key))
        new_in = und & (m2 == key)
        new_out = und & ~new_in & ((m2 >> 61) == 2)
        state[new_in] = 2
        state[new_out] = 0
    is_root = state == 2
    roots = np.flatnonzero(is_root)
    n_agg = roots.size
    agg = np.full(n, -1, np.int64)
    agg[roots] = np.arange(n_agg)
    # phase 1: join the adjacent root of largest priority
    rk = np.where(is_root, prio, -1)
    m = _max_nbr(G, rk)
    sel = ~isolated & ~is_root & (m >= 0)
    agg[sel] = agg[m[sel] & IDX_MASK]
    # phase 2: join the aggregate (largest root priority) of an assigned
    # neighbour, synchronous sweeps
    root_of = np.full(n, -1, np.int64)
    root_of[agg >= 0] = roots[agg[agg >= 0]]
    while True:
        todo = ~isolated & (agg < 0)
        if not todo.any():
            break
        rk2 = np.where(agg >= 0, prio[np.maximum(root_of, 0)], -1)
        m = _max_nbr(G, rk2)
        sel = todo & (m >= 0)
        if not sel.any():
            raise RuntimeError("aggregation left unreachable nodes")
        agg[sel] = agg[m[sel] & IDX_MASK]
        root_of[sel] = roots[agg[sel]]
    if return_roots:
        return agg, n_agg, roots
    return agg, n_agg


def mgs2_qr(Ba, drop_tol):
    """Thin QR of one aggregate block by modified Gram-Schmidt applied twice.
    A column whose remaining norm is <= drop_tol * (largest column norm) is
    dependent and dropped.  Returns ``(Q (m x r), R (r x nb))`` with
    ``diag(R) > 0``."""
    m, nb = Ba.shape
    scale = np.sqrt((Ba * Ba).sum(axis=0)).max()
    Q: List[np.ndarray] = []
    R = np.zeros((nb, nb))
    for j in range(nb):
        v = Ba[:, j].copy()
        for _ in range(2):
            for k, q in enumerate(Q):
                c = float(q @ v)
                R[k, j] += c
                v -= c * q
        nv = float(np.sqrt(v @ v))
        if nv > drop_tol * scale:
            R[len(Q), j] = nv
            Q.append(v / nv)
    r = len(Q)
    Qm = np.stack(Q, axis=1) if r else np.zeros((m, 0))
    return Qm, R[:r].copy()


def tentative_prolongator(agg, n_agg, node_ptr, B, drop_tol):
    """Block-diagonal P_tent and the coarse near-nullspace (stacked R)."""
    n_dofs, nb = B.shape
    members = np.argsort(np.where(agg >= 0, agg, n_agg), kind="stable")
    counts = np.bincount(agg[agg >= 0], minlength=n_agg)
    starts = np.r_[0, np.cumsum(counts)]
    rows, cols, vals, Rs, ranks = [], [], [], [], np.zeros(n_agg, np.int64)
    coff = 0
    for a in range(n_agg):
        nodes = members[starts[a]:starts[a + 1]]
        dofs = np.concatenate([np.arange(node_ptr[i], node_ptr[i + 1])
                               for i in nodes])
        Q, R = mgs2_qr(B[dofs], drop_tol)
        r = Q.shape[1]
        ranks[a] = r
        rr, cc = np.meshgrid(dofs, coff + np.arange(r), indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(Q.ravel())
        Rs.append(R)
        coff += r
    P = sp.csr_matrix((np.concatenate(vals),
                       (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n_dofs, coff))
    P.sort_indices()
    Bc = np.concatenate(Rs, axis=0) if Rs else np.zeros((0, nb))
    return P, Bc, ranks


def power_lambda(A, dinv, node_ptr, key_stride, its):
    """Largest eigenvalue estimate of D^{-1} A: ``its`` power iterations from
    the hashed start vector x[(a, c)] = hash_unit(stride a + c)."""
    n_nodes = node_ptr.size - 1
    cnt = np.diff(node_ptr)
    node = np.repeat(np.arange(n_nodes), cnt)
    comp = np.arange(node_ptr[-1]) - node_ptr[node]
    x = hash_unit(key_stride * node + comp)
    x = x / np.sqrt(x @ x)
    lam = 0.0
    for _ in range(its):
        y = dinv * (A @ x)
        lam = float(np.sqrt(y @ y))
        x = y / lam
    return lam


def chebyshev(A, dinv, b, x, theta, delta, degree):
    """Chebyshev iteration on D^{-1} A x = D^{-1} b (Saad, Alg. 12.1).

    ``x = None`` means a zero initial guess (no product needed for the
    first residual)."""
    if x is None:
        x = np.zeros_like(b)
        r = dinv * b
    else:
        r = dinv * (b - A @ x)
    sigma = theta / delta
    rho = 1.0 / sigma
    d = r / theta
    for k in range(degree):
        x = x + d
        if k == degree - 1:
            break
        r = r - dinv * (A @ d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * r
        rho = rho_new
    return x


class Hierarchy:
    def __init__(self, levels, opts):
        self.levels = levels
        self.opts = opts
        Ac = levels[-1].A.toarray()
        self.coarse_lu = sla.lu_factor(Ac)

    @property
    def n_levels(self):
        return len(self.levels)

    def vcycle(self, b, transpose=False, lvl=0):
        """One V(2,2) cycle ``x = AMG(K, b)``.  ``transpose`` applies the
        transposed operator: the same cycle on A_l^T (same P, R = P^T, same
        Chebyshev coefficients), the transposed coarse solve."""
        L = self.levels[lvl]
        if lvl == len(self.levels) - 1:
            return sla.lu_solve(self.coarse_lu, b, trans=1 if transpose else 0)
        A = L.AT if transpose else L.A
        deg = self.opts.cheb_degree
        x = chebyshev(A, L.dinv, b, None, L.theta, L.delta, deg)
        r = b - A @ x
        e = self.vcycle(L.R @ r, transpose, lvl + 1)
        x = x + L.P @ e
        return chebyshev(A, L.dinv, b, x, L.theta, L.delta, deg)

    def operator_complexity(self):
        nnz0 = self.levels[0].A.nnz
        return sum(L.A.nnz for L in self.levels) / nnz0


def build_hierarchy(K, pattern, coords=None, opts: Optional[AMGOptions] = None):
    """Smoothed-aggregation setup on the scalar matrix ``K`` with 3 dofs per
    node and structural node pattern ``pattern``."""
    opts = opts or AMGOptions()
    K = sp.csr_matrix(K)
    n = K.shape[0]
    B = rigid_modes(coords, n)
    nb = B.shape[1]
    node_ptr = 3 * np.arange(n // 3 + 1, dtype=np.int64)
    levels: List[Level] = []
    A, pat, stride = K, sp.csr_matrix(pattern), 3
    while True:
        L = Level(A=A, pattern=pat, node_ptr=node_ptr, key_stride=stride, B=B)
        L.dinv = 1.0 / A.diagonal()
        L.AT = sp.csr_matrix(A.T)
        levels.append(L)
        if A.shape[0] <= opts.max_coarse or len(levels) == opts.max_levels:
            break
        agg, n_agg = mis2_aggregate(pat)
        if n_agg == 0:
            break
        L.agg, L.n_agg = agg, n_agg
        lam = power_lambda(A, L.dinv, node_ptr, stride, opts.power_its)
        L.lam_hi = opts.lam_safety * lam
        lo = L.lam_hi / opts.cheb_ratio
        L.theta = 0.5 * (L.lam_hi + lo)
        L.delta = 0.5 * (L.lam_hi - lo)
        Pt, Bc, ranks = tentative_prolongator(agg, n_agg, node_ptr, B,
                                              opts.drop_tol)
        L.P_tent, L.rank = Pt, ranks
        omega = opts.omega_factor / L.lam_hi
        AP = A @ Pt
        P = sp.csr_matrix(Pt - sp.diags(omega * L.dinv) @ AP)
        P.sort_indices()
        L.P = P
        L.R = sp.csr_matrix(P.T)
        L.R.sort_indices()
        Ac = sp.csr_matrix(L.R @ (A @ P))
        Ac.sort_indices()
        # structural patterns at node level
        ptent_pat = sp.csr_matrix(
            (np.ones(int((agg >= 0).sum()), np.int8),
             (np.flatnonzero(agg >= 0), agg[agg >= 0])),
            shape=(L.n_nodes, n_agg))
        patP = bool_product(pat, ptent_pat)
        patAc = bool_product(bool_product(sp.csr_matrix(patP.T), pat), patP)
        patAc.sort_indices()
        A, pat, B, stride = Ac, patAc, Bc, nb
        node_ptr = np.r_[0, np.cumsum(ranks)].astype(np.int64)
    return Hierarchy(levels, opts)
