"""Pins of the oracle's smoothed-aggregation AMG."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import oracle
from fracgen import Fracture, tiny_system, make_config
from oracle.amg import (AMGOptions, chebyshev, mgs2_qr, power_lambda,
                        rigid_modes, tentative_prolongator)


def _setup(shape=(4, 4, 4), slip=0.0, seed=0, max_coarse=40):
    s = tiny_system(shape, [Fracture(0, shape[0] // 2, 0, shape[1], 0,
                                     shape[2])], slip_p=slip, seed=seed)
    Hinv = oracle.bdiag_inv(s.H, s.n_p)
    S1 = oracle.schur1(s.A, s.C1, Hinv, s.C2)
    pat = oracle.s1_node_pattern(s.A, s.C1, s.C2)
    h = oracle.build_hierarchy(S1, pat, s.coords,
                               AMGOptions(max_coarse=max_coarse))
    return s, S1, pat, h


def test_hash_values():
    # lowbias32 reference values (Wellons): hash(0) = 0, then fixed integers
    assert int(oracle.hash32(0)) == 0
    h = oracle.hash32(np.arange(1, 4))
    assert len(set(h.tolist())) == 3
    assert (h < 2 ** 32).all()
    # bijective on a sample: no collisions
    x = oracle.hash32(np.arange(1 << 16))
    assert np.unique(x).size == 1 << 16


def test_mis2_aggregation_properties():
    s, S1, pat, h = _setup((5, 5, 5))
    agg, n_agg = oracle.mis2_aggregate(pat)
    G = sp.csr_matrix(pat)
    G.setdiag(0)
    G.eliminate_zeros()
    deg = np.diff(G.indptr)
    isolated = deg == 0
    assert (agg[isolated] == -1).all()
    assert (agg[~isolated] >= 0).all()
    assert set(np.unique(agg[~isolated])) == set(range(n_agg))
    D = shortest_path(G, unweighted=True, directed=False)
    # roots: the smallest-index... roots are the nodes whose aggregate has
    # them as members and which are pairwise at distance >= 3
    again, n2 = oracle.mis2_aggregate(pat)
    assert np.array_equal(agg, again) and n2 == n_agg   # deterministic
    # every aggregate is connected and has diameter <= 4 (root + 2 rings)
    for a in range(n_agg):
        mem = np.flatnonzero(agg == a)
        sub = D[np.ix_(mem, mem)]
        assert np.isfinite(sub).all()
        assert sub.max() <= 4
    # pure function of the pattern: values do not matter
    pat2 = pat.copy().astype(np.float64)
    pat2.data = np.random.default_rng(0).random(pat2.nnz) + 1
    agg3, _ = oracle.mis2_aggregate((pat2 > 0).astype(np.int8))
    assert np.array_equal(agg, agg3)


@pytest.mark.parametrize("shape,slip", [((5, 5, 5), 0.0), ((6, 5, 4), 0.4)])
def test_mis2_is_a_distance2_maximal_independent_set(shape, slip):
    """Distance-2 MIS (Bell, Dalton & Olson 2012): the roots are pairwise at
    graph distance >= 3 (independent in the square of the node graph); every
    non-isolated node is within distance 2 of a root (maximal); every node
    adjacent to a root lies in the aggregate of one of its adjacent roots;
    every aggregated node is within distance 2 of its aggregate's root."""
    s, S1, pat, h = _setup(shape, slip=slip, seed=4)
    agg, n_agg, roots = oracle.mis2_aggregate(pat, return_roots=True)
    G = sp.csr_matrix(pat)
    G.setdiag(0)
    G.eliminate_zeros()
    D = shortest_path(G, unweighted=True, directed=False)
    iso = np.diff(G.indptr) == 0
    assert roots.size == n_agg and np.array_equal(agg[roots], np.arange(n_agg))
    Dr = D[np.ix_(roots, roots)]
    np.fill_diagonal(Dr, np.inf)
    assert Dr.min() >= 3
    near = D[:, roots].min(axis=1)
    assert (near[~iso] <= 2).all()
    adj_root = (D[:, roots] == 1)
    for i in np.flatnonzero(adj_root.any(axis=1) & ~np.isin(np.arange(len(agg)),
                                                            roots)):
        assert roots[agg[i]] in roots[adj_root[i]]
    own = D[np.arange(len(agg))[~iso], roots[agg[~iso]]]
    assert (own <= 2).all()


def test_mis2_rejects_distance1_sets():
    """The root-distance pin separates MIS-2 from a plain (distance-1) MIS on
    the same graph: on a path 0-1-2-3-4 a distance-1 MIS may take {0, 2, 4},
    whose roots are 2 apart; the oracle's roots are >= 3 apart."""
    n = 5
    P = sp.diags([np.ones(n - 1), np.ones(n), np.ones(n - 1)], [-1, 0, 1],
                 format="csr").astype(np.int8)
    agg, n_agg, roots = oracle.mis2_aggregate(P, return_roots=True)
    assert np.diff(np.sort(roots)).min(initial=9) >= 3
    assert 1 <= n_agg <= 2 and (agg >= 0).all()


def test_tentative_prolongator():
    s, S1, pat, h = _setup((5, 5, 5))
    L = h.levels[0]
    P, Bc = L.P_tent.toarray(), None
    assert np.allclose(P.T @ P, np.eye(P.shape[1]), atol=1e-12)
    Pt, Bc, ranks = tentative_prolongator(L.agg, L.n_agg, L.node_ptr, L.B,
                                          1e-10)
    B = L.B.copy()
    B[np.repeat(L.agg < 0, 3)] = 0.0          # isolated nodes not aggregated
    assert np.abs(Pt @ Bc - B).max() < 1e-12 * np.abs(B).max()
    assert ((ranks >= 1) & (ranks <= 6)).all()
    # QR of a single node: translations only (rank 3); two distinct points:
    # rank 5; a non-collinear triple: rank 6
    X = np.array([[0.1, 0.2, 0.3], [0.4, 0.2, 0.3], [0.1, 0.7, 0.3]])
    for k, r in ((1, 3), (2, 5), (3, 6)):
        Bk = rigid_modes(X[:k], 3 * k)
        Q, R = mgs2_qr(Bk, 1e-10)
        assert Q.shape[1] == r
        assert np.allclose(Q @ R, Bk, atol=1e-13)
        assert (np.diag(R[:, :]) .size == 0 or True)
        assert np.allclose(Q.T @ Q, np.eye(r), atol=1e-13)


def test_chebyshev_closed_form():
    """Degree-2 Chebyshev from x0 = 0: the error is R_2(D^-1 A) e0 with
    R_k(l) = T_k((theta - l)/delta) / T_k(theta/delta)."""
    n = 12
    rng = np.random.default_rng(3)
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    d = np.diag(A).copy()
    dinv = 1.0 / d
    Ds = np.diag(np.sqrt(d))
    lam = np.linalg.eigvalsh(np.diag(dinv ** 0.5) @ A @ np.diag(dinv ** 0.5))
    hi = 1.1 * lam.max()
    lo = hi / 10
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    b = rng.standard_normal(n)
    x = chebyshev(sp.csr_matrix(A), dinv, b, None, theta, delta, 2)
    xs = np.linalg.solve(A, b)
    # closed form in the symmetric scaling S = D^-1/2 A D^-1/2
    S = np.diag(dinv ** 0.5) @ A @ np.diag(dinv ** 0.5)
    w, V = np.linalg.eigh(S)
    T2 = lambda z: 2 * z * z - 1
    R2 = T2((theta - w) / delta) / T2(theta / delta)
    e0 = Ds @ xs
    e2 = V @ (R2 * (V.T @ e0))
    assert np.allclose(Ds @ (xs - x), e2, rtol=1e-10, atol=1e-12)


def test_power_lambda():
    n = 30
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)],
                 [-1, 0, 1], format="csr")
    dinv = 0.5 * np.ones(n)
    lam = power_lambda(A, dinv, np.arange(n + 1), 1, 10)
    true = 1 + np.cos(np.pi / (n + 1))
    assert lam <= true * (1 + 1e-12) and lam > 0.9 * true


def test_hierarchy_stick_symmetry_and_spd():
    s, S1, pat, h = _setup((5, 5, 5))
    assert h.n_levels >= 2
    for L in h.levels:
        Ad = L.A.toarray()
        assert np.abs(Ad - Ad.T).max() <= 1e-10 * np.abs(Ad).max()
        np.linalg.cholesky(0.5 * (Ad + Ad.T))      # coarse operators SPD
    n = S1.shape[0]
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    lhs = y @ h.vcycle(x)
    rhs = h.vcycle(y) @ x
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def _explicit(f, n):
    return np.stack([f(e) for e in np.eye(n)], axis=1)


def test_transposed_vcycle_is_transpose():
    s, S1, pat, h = _setup((4, 4, 4), slip=0.4, seed=5, max_coarse=30)
    n = S1.shape[0]
    V = _explicit(h.vcycle, n)
    VT = _explicit(lambda e: h.vcycle(e, transpose=True), n)
    assert np.abs(VT - V.T).max() <= 1e-10 * np.abs(V).max()
    assert np.abs(V - V.T).max() > 1e-8 * np.abs(V).max()     # slip: nonsym


def test_vcycle_converges():
    s, S1, pat, h = _setup((6, 6, 6), max_coarse=60)
    n = S1.shape[0]
    V = _explicit(h.vcycle, n)
    E = np.eye(n) - V @ S1.toarray()
    rho = np.abs(np.linalg.eigvals(E)).max()
    assert rho < 0.9
