"""Pins of the oracle's block surrogates (Sec. 3, Alg 3.1 and 3.3)."""
import numpy as np
import pytest
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


def test_fixed_stress_diagonal_and_hand_case():
    """eq. FS_algebraic pinned without retyping it.  (1) With a diagonal D in
    place of S1 every principal submatrix is diagonal, so
    [S_K]_k = (Q2 D^{-1} Q1)_kk exactly.  (2) A 3-dof, 2-face case worked by
    hand: S1 = [[2,1,0],[1,3,1],[0,1,4]], Q1 columns (1,2,0) and (0,1,3),
    Q2 rows (1,1,0) and (1,0,0).  Face 0: K = {0,1}, S1^(0) = [[2,1],[1,3]],
    (1,1) S1^(0)^-1 (1,2) = 4/5.  Face 1: K = {1,2} U {0} = all three dofs,
    e_0^T S1^{-1} (0,1,3) = (11, -4, 1)/18 . (0,1,3) = -1/18 (restricting
    to nz(Q1 col) alone would give 0)."""
    s = _sys()
    Q2 = _random_q2(s, seed=3, density=0.7)
    rng = np.random.default_rng(1)
    d = rng.random(s.n_u) + 0.5
    D = sp.diags(d, format="csr")
    fs = oracle.fixed_stress(D, s.Q1, Q2)
    ref = (Q2 @ sp.diags(1.0 / d) @ s.Q1).diagonal()
    assert np.allclose(fs, ref, rtol=1e-13, atol=0)
    assert (fs != 0).any()
    S1 = sp.csr_matrix(np.array([[2.0, 1, 0], [1, 3, 1], [0, 1, 4]]))
    Q1 = sp.csr_matrix(np.array([[1.0, 0], [2, 1], [0, 3]]))
    Q2h = sp.csr_matrix(np.array([[1.0, 1, 0], [1, 0, 0]]))
    fs = oracle.fixed_stress(S1, Q1, Q2h)
    assert np.allclose(fs, [4.0 / 5.0, -1.0 / 18.0], rtol=1e-14, atol=0)


def _psi_and_fu_action(s, v, eps=1e-7):
    """Psi(Q1^T) v (the rows of Q1^T v on open faces) and F_u v, the
    directional derivative of the TPFA flux part of the pressure residual
    (eq. FV_inner_product with the cubic law on open faces) by central
    differences, built without the generator's Q2."""
    from fracgen.problem import assemble_T
    area = s.h * s.h
    g0 = s.extras["aperture"]
    opn = s.face_state == 2
    psi = np.where(opn, s.Q1.T @ v, 0.0)

    def flux(u):
        g = g0 - (s.Q1.T @ u) / area
        ups = np.where(opn, s.upsilon * (g / g0) ** 3, s.upsilon)
        return assemble_T(s, ups) @ s.extras["p_state"]
    fu = (flux(eps * v) - flux(-eps * v)) / (2 * eps)
    return psi, fu


@pytest.mark.parametrize("name", ["tiny_open", "c1o"])
def test_schur_tpu_open_faces_relation(name):
    """The t-p-u Schur surrogate with open faces against the relation the
    paper states after the remark on S~2 (Sec. 3.2):
    S~ = S1 + (1/dt) Q1 T~^{-1} Psi(Q1^T) - Q1 T~^{-1} F_u, T~ = diag(T),
    with Psi and F_u formed independently of Q2 (F_u by central differences
    of the flux residual).  A wrong sign, T in place of diag(T) or a dropped
    term changes the action by O(1)."""
    import fracgen
    from fracgen.problem import DT
    if name == "tiny_open":
        s = fracgen.tiny_system((4, 4, 4), slip_p=0.3, open_p=0.4, seed=3)
    else:
        s = fracgen.make_config(name)
    assert s.Q2.nnz > 0
    Hinv = oracle.bdiag_inv(s.H, s.n_p)
    S1 = oracle.schur1(s.A, s.C1, Hinv, s.C2)
    St = oracle.schur_tpu(s.A, s.C1, Hinv, s.C2, s.Q1, s.T, s.Q2)
    tdi = 1.0 / s.T.diagonal()
    rng = np.random.default_rng(7)
    for _ in range(3):
        v = rng.standard_normal(s.n_u)
        v[s.dirichlet] = 0.0
        psi, fu = _psi_and_fu_action(s, v)
        rel = s.Q1 @ (tdi * psi) / DT - s.Q1 @ (tdi * fu)
        got = St @ v - S1 @ v
        assert np.linalg.norm(rel) > 1e-6 * np.linalg.norm(S1 @ v)
        assert np.linalg.norm(got - rel) <= 1e-6 * np.linalg.norm(rel)


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
