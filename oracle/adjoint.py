"""Adjoint gradients of a fracture-pressure misfit.

For ``J x = b`` and a loss ``L(x)``, the adjoint ``J^T lam = dL/dx`` gives
``dL/db = lam`` and ``dL/dtheta = -lam^T (dJ/dtheta) x``.  With ``theta_K =
log Upsilon_K`` only the pressure block ``T`` depends on theta: through the
TPFA transmissibilities ``Upsilon_KL = 2 U_K U_L / (U_K + U_L)`` (harmonic
average, eq. FV_inner_product) and the Dirichlet terms ``U_K``.  So

    dL/dtheta_K = - sum_{edges KL} dU_KL/dtheta_K (lam_K - lam_L)(p_K - p_L)
                  - ndir_K U_K lam_K p_K,
    dU_KL/dtheta_K = 2 U_K U_L^2 / (U_K + U_L)^2.

The finite-difference reference evaluates the loss in 80-bit extended
precision: with no open faces (Q2 = 0) the pressure row decouples, ``p =
T^{-1} b_p`` exactly, and T is factored per connected component by a
banded Cholesky in ``numpy.longdouble``.
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


def loss_and_grad_x(x, n_u, n_t, p_obs):
    """L = 0.5 |p - p_obs|^2 and dL/dx = [0; 0; p - p_obs]."""
    p = x[n_u + n_t:]
    r = p - p_obs
    g = np.zeros_like(x)
    g[n_u + n_t:] = r
    return 0.5 * float(r @ r), g


def grad_log_trans(pairs, ndir, upsilon, lam_p, p):
    """Edge-wise dL/d(log Upsilon) from the adjoint pressure ``lam_p``."""
    K, L = pairs[:, 0], pairs[:, 1]
    uK, uL = upsilon[K], upsilon[L]
    s = uK + uL
    dK = 2.0 * uK * uL * uL / (s * s)
    dL = 2.0 * uL * uK * uK / (s * s)
    jump = (lam_p[K] - lam_p[L]) * (p[K] - p[L])
    n = upsilon.size
    g = -(np.bincount(K, dK * jump, n) + np.bincount(L, dL * jump, n))
    g -= ndir * upsilon * lam_p * p
    return g


# ----------------------------------------------------------------------------
# extended-precision finite differences
# ----------------------------------------------------------------------------

def _T_ld(pairs, ndir, ups, T_stab, faces):
    """Dense longdouble T on the face subset ``faces`` (a union of
    components): TPFA + Dirichlet + j_p/dt."""
    ld = np.longdouble
    loc = -np.ones(ups.size, np.int64)
    loc[faces] = np.arange(faces.size)
    n = faces.size
    T = np.zeros((n, n), dtype=ld)
    Ts = sp.csr_matrix(T_stab)[faces][:, faces].toarray().astype(ld)
    T += Ts
    sel = (loc[pairs[:, 0]] >= 0) & (loc[pairs[:, 1]] >= 0)
    for K, L in pairs[sel]:
        uK, uL = ld(ups[K]), ld(ups[L])
        w = ld(2) * uK * uL / (uK + uL)
        i, j = loc[K], loc[L]
        T[i, i] += w
        T[j, j] += w
        T[i, j] -= w
        T[j, i] -= w
    for K in faces:
        T[loc[K], loc[K]] += ld(ndir[K]) * ld(ups[K])
    return T


def _chol_solve_ld(M, rhs):
    """Banded Cholesky solve in longdouble (band taken from M)."""
    n = M.shape[0]
    nz = np.nonzero(M)
    bw = int(np.max(np.abs(nz[0] - nz[1]))) if n else 0
    L = M.copy()
    for k in range(n):
        if L[k, k] <= 0:
            raise np.linalg.LinAlgError("not SPD")
        L[k, k] = np.sqrt(L[k, k])
        e = min(n, k + bw + 1)
        L[k + 1:e, k] /= L[k, k]
        L[k + 1:e, k + 1:e] -= np.outer(L[k + 1:e, k], L[k + 1:e, k])
    y = np.zeros(n, dtype=M.dtype)
    for k in range(n):
        s0 = max(0, k - bw)
        y[k] = (rhs[k] - L[k, s0:k] @ y[s0:k]) / L[k, k]
    x = np.zeros(n, dtype=M.dtype)
    for k in range(n - 1, -1, -1):
        e = min(n, k + bw + 1)
        x[k] = (y[k] - L[k + 1:e, k] @ x[k + 1:e]) / L[k, k]
    return x


def fd_grad_log_trans(pairs, ndir, upsilon, T_stab, b_p, p_obs, faces,
                      h=1e-6):
    """Central differences of L = 0.5 |T(U)^{-1} b_p - p_obs|^2 with respect
    to log U_K for each K in ``faces``, in 80-bit precision."""
    n = upsilon.size
    G = sp.csr_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])),
                      shape=(n, n))
    ncomp, lab = connected_components(G, directed=False)
    ld = np.longdouble
    out = np.zeros(len(faces))
    for i, K in enumerate(faces):
        comp = np.flatnonzero(lab == lab[K])
        vals = []
        for sgn in (1, -1):
            ups = upsilon.astype(ld).copy()
            ups[K] = ups[K] * np.exp(ld(sgn) * ld(h))
            T = _T_ld(pairs, ndir, ups, T_stab, comp)
            p = _chol_solve_ld(T, b_p[comp].astype(ld))
            r = p - p_obs[comp].astype(ld)
            vals.append(ld(0.5) * (r @ r))
        out[i] = float((vals[0] - vals[1]) / (ld(2) * ld(h)))
    return out
