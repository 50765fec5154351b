"""Block surrogates and Schur complements of the block preconditioners.

* ``H~ = Bdiag(H, 3)``                       Alg 3.1 / 3.3, first step
* ``S1 = A + C1 H~^{-1} C2``                 eq. Schur1_2, Alg 3.3 step 2
* ``S~ = A + C1 H~^{-1} C2 - Q1 T~^{-1} Q2``  eq. appSchur_1, Alg 3.1 step 3
* ``S_K = FS(Q2, S1, Q1)``                   eq. Ak and eq. FS_algebraic
"""
import numpy as np
import scipy.sparse as sp


def bdiag_inv(H, n_p):
    """Inverses of the ``n_p`` 3x3 diagonal face blocks of ``H`` (H~ = Bdiag(H,3),
    Sec. 3.1).  Returns an ``(n_p, 3, 3)`` array; raises on a singular block."""
    H = sp.csr_matrix(H)
    blk = np.zeros((n_p, 3, 3))
    base = 3 * np.arange(n_p)
    for r in range(3):
        for c in range(3):
            blk[:, r, c] = np.asarray(H[base + r, base + c]).ravel()
    det = np.linalg.det(blk)
    if np.any(det == 0) or not np.all(np.isfinite(det)):
        raise np.linalg.LinAlgError("singular face block in Bdiag(H,3)")
    return np.linalg.inv(blk)


def bdiag_matrix(blocks):
    """Sparse block-diagonal matrix from an ``(n, 3, 3)`` array."""
    n = blocks.shape[0]
    return sp.bsr_matrix((blocks, np.arange(n), np.arange(n + 1)),
                         shape=(3 * n, 3 * n)).tocsr()


def bdiag_apply(blocks, v, transpose=False):
    """``Bdiag^{-1} v`` (or its transpose) face by face."""
    V = np.asarray(v).reshape(-1, 3)
    if transpose:
        return np.einsum("kji,kj->ki", blocks, V).ravel()
    return np.einsum("kij,kj->ki", blocks, V).ravel()


def schur1(A, C1, Hinv, C2):
    """First-level Schur complement ``S1 = A + C1 H~^{-1} C2`` (eq. Schur1_2)."""
    return sp.csr_matrix(A + C1 @ (bdiag_matrix(Hinv) @ C2))


def schur_tpu(A, C1, Hinv, C2, Q1, T, Q2):
    """t-p-u Schur surrogate ``S~ = A + C1 H~^{-1} C2 - Q1 T~^{-1} Q2`` with
    ``T~ = diag(T)`` (eq. appSchur_1, Alg 3.1)."""
    S = schur1(A, C1, Hinv, C2)
    if Q2.nnz:
        Tt = sp.diags(1.0 / T.diagonal())
        S = sp.csr_matrix(S - Q1 @ (Tt @ Q2))
    return S


def fixed_stress(S1, Q1, Q2):
    """Algebraic fixed-stress diagonal (Remark on eq. FS, eqs. Ak and
    FS_algebraic): for face k, K^(k) = nz(Q1 column k) U nz(Q2 row k),
    S1^(k) the principal submatrix of S1 on K^(k), and
    [S_K]_k = Q2^(k)^T S1^(k)^{-1} Q1^(k)."""
    n_p = Q1.shape[1]
    out = np.zeros(n_p)
    if Q2.nnz == 0:
        return out
    Q1c = sp.csc_matrix(Q1)
    Q2r = sp.csr_matrix(Q2)
    S1 = sp.csr_matrix(S1)
    for k in range(n_p):
        k2 = Q2r.indices[Q2r.indptr[k]:Q2r.indptr[k + 1]]
        if k2.size == 0:
            continue
        k1 = Q1c.indices[Q1c.indptr[k]:Q1c.indptr[k + 1]]
        K = np.union1d(k1, k2)
        Sk = S1[K][:, K].toarray()
        q1 = np.asarray(Q1c[K, k].todense()).ravel()
        q2 = np.asarray(Q2r[k, K].todense()).ravel()
        out[k] = q2 @ np.linalg.solve(Sk, q1)
    return out


def node_pattern(M, br, bc):
    """Boolean block pattern of ``M`` for row / column block sizes br, bc."""
    M = sp.coo_matrix(M)
    nr = -(-M.shape[0] // br)
    nc = -(-M.shape[1] // bc)
    P = sp.csr_matrix((np.ones(M.nnz, np.int8), (M.row // br, M.col // bc)),
                      shape=(nr, nc))
    P.sum_duplicates()
    P.data[:] = 1
    return P


def bool_product(P, Q):
    R = sp.csr_matrix(P.astype(np.int64) @ Q.astype(np.int64))
    R.data[:] = 1
    return R.astype(np.int8)


def s1_node_pattern(A, C1, C2):
    """Structural node-level pattern of S1: pattern(A) U pattern(C1) pattern(C2)
    over 3x3 node / face blocks (no numerical cancellation)."""
    PA = node_pattern(A, 3, 3)
    P = bool_product(node_pattern(C1, 3, 3), node_pattern(C2, 3, 3))
    R = sp.csr_matrix(PA.astype(np.int64) + P.astype(np.int64))
    R.data[:] = 1
    R.sort_indices()
    return R.astype(np.int8)
