"""Pins of the oracle's block surrogates (Sec. 3, Alg 3.1 and 3.3)."""
import numpy as np
import scipy.sparse as sp

import oracle
from fracgen import Fracture, tiny_system
from oracle.blocks import node_pattern


def _sys(slip=0.0, seed=0):
    return tiny_system((4, 4, 4), [Fracture(0, 2, 0, 4, 0, 4),
                                   Fracture(2, 2, 0, 4, 0, 4)],
                       slip_p=slip, seed=seed)


def _random_q2(s, seed=0, density=1.0):
    """A synthetic non-empty Q2 with the pattern of Q1^T (open-face like)."""
    rng = np.random.default_rng(seed)
    Q = sp.csr_matrix(s.Q1.T).copy()
    Q.data = rng.standard_normal(Q.nnz) * np.abs(Q.data).max() * 0.3
    keep = rng.random(s.n_p) < density
    Q = sp.diags(keep.astype(float)) @ Q
    Q = sp.csr_matrix(Q)
    Q.eliminate_zeros()
    return Q


def test_bdiag_inverse():
    s = _sys(slip=0.5, seed=2)
    Hinv = oracle.bdiag_inv(s.H, s.n_p)
    H = s.H.toarray()
    for K in range(s.n_p):
        blk = H[3 * K:3 * K + 3, 3 * K:3 * K + 3]
        assert np.allclose(Hinv[K] @ blk, np.eye(3), atol=1e-12)
    v = np.random.default_rng(0).standard_normal(s.n_t)
    assert np.allclose(oracle.bdiag_apply(Hinv, v),
                       oracle.bdiag_matrix(Hinv) @ v, rtol=1e-14)
    assert np.allclose(oracle.bdiag_apply(Hinv, v, transpose=True),
                       oracle.bdiag_matrix(Hinv).T @ v, rtol=1e-14)


def test_schur_and_pattern():
    s = _sys(slip=0.3, seed=1)
    Hinv = oracle.bdiag_inv(s.H, s.n_p)
    S1 = oracle.schur1(s.A, s.C1, Hinv, s.C2).toarray()
    # dense definition with the explicitly inverted face blocks
    Hd = s.H.toarray()
    Hb = np.zeros_like(Hd)
    for K in range(s.n_p):
        sl = slice(3 * K, 3 * K + 3)
        Hb[sl, sl] = np.linalg.inv(Hd[sl, sl])
    ref = s.A.toarray() + s.C1.toarray() @ Hb @ s.C2.toarray()
    assert np.abs(S1 - ref).max() <= 1e-12 * np.abs(ref).max()
    # structural node pattern covers every numerical nonzero
    pat = oracle.s1_node_pattern(s.A, s.C1, s.C2).toarray() > 0
    num = node_pattern(sp.csr_matrix(ref), 3, 3).toarray() > 0
    assert not (num & ~pat).any()
    assert pat.diagonal().all()
    # Q2 = 0: the t-p-u surrogate equals S1 (eq. S-S1 relation, Psi = F_u = 0)
    St = oracle.schur_tpu(s.A, s.C1, Hinv, s.C2, s.Q1, s.T, s.Q2).toarray()
    assert np.array_equal(St, S1)


def test_s1_definiteness():
    """Remark after Prop 3.2: S1 is SPD in stick; with slip faces it is
    non-symmetric with its spectrum in the right half-plane."""
    s = _sys()
    Hinv = oracle.bdiag_inv(s.H, s.n_p)
    S1 = oracle.schur1(s.A, s.C1, Hinv, s.C2).toarray()
    assert np.allclose(S1, S1.T, rtol=0, atol=1e-12 * np.abs(S1).max())
    np.linalg.cholesky(0.5 * (S1 + S1.T))
    for seed in range(3):
        s = _sys(slip=0.3, seed=seed)
        Hinv = oracle.bdiag_inv(s.H, s.n_p)
        S1 = oracle.schur1(s.A, s.C1, Hinv, s.C2).toarray()
        assert not np.allclose(S1, S1.T)
        ev = np.linalg.eigvals(S1)
        assert ev.real.min() > 0


def test_fixed_stress():
    s = _sys()
    Hinv = oracle.bdiag_inv(s.H, s.n_p)
    S1 = oracle.schur1(s.A, s.C1, Hinv, s.C2)
    assert not oracle.fixed_stress(S1, s.Q1, s.Q2).any()
    Q2 = _random_q2(s, density=0.6)
    fs = oracle.fixed_stress(S1, s.Q1, Q2)
    S1d, Q1d, Q2d = S1.toarray(), s.Q1.toarray(), Q2.toarray()
    for k in range(s.n_p):
        K = np.union1d(np.flatnonzero(Q1d[:, k]), np.flatnonzero(Q2d[k]))
        exp = Q2d[k, K] @ np.linalg.solve(S1d[np.ix_(K, K)], Q1d[K, k])
        assert np.isclose(fs[k], exp, rtol=1e-12, atol=1e-300)
    assert (fs != 0).any()
