"""Pins of the block preconditioners against the paper's algebra.

* step-by-step Alg 3.2 / 3.4 versus the inverse of the inexact block LDU
  factorizations (eq. LDU1 / eq. LDU2), built independently here,
* the transposed application is the transpose,
* exactness when H is block diagonal, Q2 = 0 and the inner solves exact,
* Prop 3.1 (n_p unit eigenvalues) and the closed forms eq. PJ_tpu and
  eq. precmat_tup,
* t-p-u and t-u-p coincide when Q2 = 0 (eq. S-S1 relation).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from fracgen import Fracture, tiny_system
from oracle.amg import AMGOptions

from test_oracle_blocks import _random_q2


def _system(q2=True, slip=0.3, seed=3):
    s = tiny_system((4, 4, 4), [Fracture(0, 2, 0, 4, 0, 4)], slip_p=slip,
                    seed=seed)
    blocks = s.blocks()
    if q2:
        blocks["Q2"] = _random_q2(s, seed=seed, density=0.5)
    return s, blocks


def _explicit(f, n):
    return np.stack([f(e) for e in np.eye(n)], axis=1)


def _pc(s, blocks, mode, inner="amg"):
    return oracle.BlockPrecond(blocks, s.n_u, s.n_t, s.n_p, mode=mode,
                               inner=inner, coords=s.coords,
                               amg_opts=AMGOptions(max_coarse=40))


def _perm(s, order):
    """Permutation matrix Q with (Q x) = x reordered into ``order``."""
    nu, nt, n_p = s.n_u, s.n_t, s.n_p
    seg = {"u": np.arange(nu), "t": nu + np.arange(nt),
           "p": nu + nt + np.arange(n_p)}
    idx = np.concatenate([seg[c] for c in order])
    Q = np.zeros((idx.size, idx.size))
    Q[np.arange(idx.size), idx] = 1.0
    return Q


def _dense_blocks(blocks):
    return {k: v.toarray() for k, v in blocks.items()}


def test_tup_matches_inverse_of_ldu2():
    s, blocks = _system()
    pc = _pc(s, blocks, "tup")
    N = s.N
    M = _explicit(pc.apply, N)
    D = _dense_blocks(blocks)
    Sinv = _explicit(pc.inner, s.n_u)           # the AMG operator
    S1t = np.linalg.inv(Sinv)                    # S~1
    Ht = np.linalg.inv(oracle.bdiag_matrix(pc.Hinv).toarray())
    S2t = pc.S2t.toarray()
    It, Iu, Ip = np.eye(s.n_t), np.eye(s.n_u), np.eye(s.n_p)
    Z = np.zeros
    L2 = np.block([[It, Z((s.n_t, s.n_u)), Z((s.n_t, s.n_p))],
                   [-D["C1"] @ np.linalg.inv(Ht), Iu, Z((s.n_u, s.n_p))],
                   [Z((s.n_p, s.n_t)), D["Q2"] @ Sinv, Ip]])
    D2 = np.block([[-Ht, Z((s.n_t, s.n_u)), Z((s.n_t, s.n_p))],
                   [Z((s.n_u, s.n_t)), S1t, Z((s.n_u, s.n_p))],
                   [Z((s.n_p, s.n_t)), Z((s.n_p, s.n_u)), S2t]])
    U2 = np.block([[It, -np.linalg.inv(Ht) @ D["C2"], Z((s.n_t, s.n_p))],
                   [Z((s.n_u, s.n_t)), Iu, Sinv @ D["Q1"]],
                   [Z((s.n_p, s.n_t)), Z((s.n_p, s.n_u)), Ip]])
    Q2p = _perm(s, "tup")
    Minv_ref = Q2p.T @ np.linalg.inv(L2 @ D2 @ U2) @ Q2p
    assert np.abs(M - Minv_ref).max() <= 1e-8 * np.abs(Minv_ref).max()
    # transposed application
    MT = _explicit(pc.apply_T, N)
    assert np.abs(MT - M.T).max() <= 1e-10 * np.abs(M).max()


def test_tup_star_matches_inverse_of_l2d2():
    """M2* (remark after Prop 3.2) is (L2 D2)^{-1} with the factors of
    eq. LDU2, and its transposed application is the transpose."""
    s, blocks = _system()
    pc = _pc(s, blocks, "tup_star")
    M = _explicit(pc.apply, s.N)
    D = _dense_blocks(blocks)
    Sinv = _explicit(pc.inner, s.n_u)
    S1t = np.linalg.inv(Sinv)
    Ht = np.linalg.inv(oracle.bdiag_matrix(pc.Hinv).toarray())
    S2t = pc.S2t.toarray()
    It, Iu, Ip = np.eye(s.n_t), np.eye(s.n_u), np.eye(s.n_p)
    Z = np.zeros
    L2 = np.block([[It, Z((s.n_t, s.n_u)), Z((s.n_t, s.n_p))],
                   [-D["C1"] @ np.linalg.inv(Ht), Iu, Z((s.n_u, s.n_p))],
                   [Z((s.n_p, s.n_t)), D["Q2"] @ Sinv, Ip]])
    D2 = np.block([[-Ht, Z((s.n_t, s.n_u)), Z((s.n_t, s.n_p))],
                   [Z((s.n_u, s.n_t)), S1t, Z((s.n_u, s.n_p))],
                   [Z((s.n_p, s.n_t)), Z((s.n_p, s.n_u)), S2t]])
    Q2p = _perm(s, "tup")
    ref = Q2p.T @ np.linalg.inv(L2 @ D2) @ Q2p
    assert np.abs(M - ref).max() <= 1e-8 * np.abs(ref).max()
    MT = _explicit(pc.apply_T, s.N)
    assert np.abs(MT - M.T).max() <= 1e-10 * np.abs(M).max()


def test_tpu_matches_inverse_of_ldu1():
    s, blocks = _system()
    pc = _pc(s, blocks, "tpu")
    M = _explicit(pc.apply, s.N)
    D = _dense_blocks(blocks)
    Sinv = _explicit(pc.inner, s.n_u)
    St = np.linalg.inv(Sinv)
    Ht = np.linalg.inv(oracle.bdiag_matrix(pc.Hinv).toarray())
    Hti = np.linalg.inv(Ht)
    T = D["T"]
    Ti = np.linalg.inv(T)
    It, Iu, Ip = np.eye(s.n_t), np.eye(s.n_u), np.eye(s.n_p)
    Z = np.zeros
    L1 = np.block([[It, Z((s.n_t, s.n_p)), Z((s.n_t, s.n_u))],
                   [Z((s.n_p, s.n_t)), Ip, Z((s.n_p, s.n_u))],
                   [-D["C1"] @ Hti, D["Q1"] @ Ti, Iu]])
    D1 = np.block([[-Ht, Z((s.n_t, s.n_p)), Z((s.n_t, s.n_u))],
                   [Z((s.n_p, s.n_t)), T, Z((s.n_p, s.n_u))],
                   [Z((s.n_u, s.n_t)), Z((s.n_u, s.n_p)), St]])
    U1 = np.block([[It, Z((s.n_t, s.n_p)), -Hti @ D["C2"]],
                   [Z((s.n_p, s.n_t)), Ip, Ti @ D["Q2"]],
                   [Z((s.n_u, s.n_t)), Z((s.n_u, s.n_p)), Iu]])
    Q1p = _perm(s, "tpu")
    Minv_ref = Q1p.T @ np.linalg.inv(L1 @ D1 @ U1) @ Q1p
    assert np.abs(M - Minv_ref).max() <= 1e-8 * np.abs(Minv_ref).max()
    MT = _explicit(pc.apply_T, s.N)
    assert np.abs(MT - M.T).max() <= 1e-10 * np.abs(M).max()


def test_exactness():
    """H block diagonal, Q2 = 0, exact inner solves: M = J^{-1} and FGMRES
    converges in one iteration."""
    for mode in ("tup", "tpu"):
        s, blocks = _system(q2=False, slip=0.3)
        Hinv = oracle.bdiag_inv(s.H, s.n_p)
        blocks["H"] = sp.csr_matrix(np.linalg.inv(
            oracle.bdiag_matrix(Hinv).toarray()))
        pc = _pc(s, blocks, mode, inner="exact")
        J = sp.bmat([[blocks["A"], blocks["C1"], blocks["Q1"]],
                     [blocks["C2"], -blocks["H"], None],
                     [blocks["Q2"], None, blocks["T"]]]).toarray()
        M = _explicit(pc.apply, s.N)
        assert np.abs(M @ J - np.eye(s.N)).max() < 1e-8
        x, info = oracle.fgmres(pc.matvec, pc.apply, s.b, rtol=1e-10)
        assert info.iterations == 1 and info.converged


def test_prop31_unit_eigenvalues_and_closed_form():
    s, blocks = _system(q2=True)
    pc = _pc(s, blocks, "tpu")
    D = _dense_blocks(blocks)
    J = sp.bmat([[blocks["A"], blocks["C1"], blocks["Q1"]],
                 [blocks["C2"], -blocks["H"], None],
                 [blocks["Q2"], None, blocks["T"]]]).toarray()
    Q1p = _perm(s, "tpu")
    M = _explicit(pc.apply, s.N)
    PJ = (Q1p @ M @ Q1p.T) @ (Q1p @ J @ Q1p.T)
    ev = np.linalg.eigvals(PJ)
    assert (np.abs(ev - 1) < 1e-6).sum() >= s.n_p
    # eq. PJ_tpu with E_H = I - H~^{-1} H and E_S = I - S~^{-1} S
    Hti = oracle.bdiag_matrix(pc.Hinv).toarray()
    Sti = _explicit(pc.inner, s.n_u)
    Ti = np.linalg.inv(D["T"])
    S = D["A"] + D["C1"] @ Hti @ D["C2"] - D["Q1"] @ Ti @ D["Q2"]
    EH = np.eye(s.n_t) - Hti @ D["H"]
    ES = np.eye(s.n_u) - Sti @ S
    C1, C2, Q2 = D["C1"], D["C2"], D["Q2"]
    Z = np.zeros
    ref = np.block([
        [np.eye(s.n_t) + (Hti @ C2 @ Sti @ C1 - np.eye(s.n_t)) @ EH,
         Z((s.n_t, s.n_p)), -Hti @ C2 @ ES],
        [-Ti @ Q2 @ Sti @ C1 @ EH, np.eye(s.n_p), Ti @ Q2 @ ES],
        [Sti @ C1 @ EH, Z((s.n_u, s.n_p)), np.eye(s.n_u) - ES]])
    assert np.abs(PJ - ref).max() <= 1e-6 * max(1.0, np.abs(ref).max())


def test_prop32_closed_form():
    s, blocks = _system(q2=True)
    pc = _pc(s, blocks, "tup")
    D = _dense_blocks(blocks)
    J = sp.bmat([[blocks["A"], blocks["C1"], blocks["Q1"]],
                 [blocks["C2"], -blocks["H"], None],
                 [blocks["Q2"], None, blocks["T"]]]).toarray()
    Q2p = _perm(s, "tup")
    M = _explicit(pc.apply, s.N)
    PJ = (Q2p @ M @ Q2p.T) @ (Q2p @ J @ Q2p.T)
    Hti = oracle.bdiag_matrix(pc.Hinv).toarray()
    S1i = _explicit(pc.inner, s.n_u)
    S2i = np.linalg.inv(pc.S2t.toarray())
    C1, C2, Q1, Q2, T, H = (D[k] for k in ("C1", "C2", "Q1", "Q2", "T", "H"))
    S1 = D["A"] + C1 @ Hti @ C2
    EH = np.eye(s.n_t) - Hti @ H
    ES1 = np.eye(s.n_u) - S1i @ S1
    S2hat = T - Q2 @ S1i @ Q1
    ES2 = np.eye(s.n_p) - S2i @ S2hat
    Iq = np.eye(s.n_u) + S1i @ Q1 @ S2i @ Q2
    It = np.eye(s.n_t)
    ref = np.block([
        [It + (-It + Hti @ C2 @ Iq @ S1i @ C1) @ EH, -Hti @ C2 @ Iq @ ES1,
         Hti @ C2 @ S1i @ Q1 @ ES2],
        [Iq @ S1i @ C1 @ EH, np.eye(s.n_u) - Iq @ ES1, S1i @ Q1 @ ES2],
        [-S2i @ Q2 @ S1i @ C1 @ EH, S2i @ Q2 @ ES1, np.eye(s.n_p) - ES2]])
    assert np.abs(PJ - ref).max() <= 1e-6 * max(1.0, np.abs(ref).max())


def test_tpu_equals_tup_without_q2():
    s, blocks = _system(q2=False)
    a = _explicit(_pc(s, blocks, "tup").apply, s.N)
    b = _explicit(_pc(s, blocks, "tpu").apply, s.N)
    assert np.abs(a - b).max() <= 1e-10 * np.abs(a).max()
