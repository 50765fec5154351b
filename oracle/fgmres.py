"""Right-preconditioned flexible GMRES(m).

The paper solves every Jacobian system with right-preconditioned full GMRES
from a zero initial guess, stopping at a 1e-8 relative residual reduction
(Sec. 4, introduction).  This oracle uses the flexible variant with restart
``m`` (Saad, SIAM J. Sci. Comput. 14 (1993)): ``z_j = M^{-1} v_j`` is stored
and the update is ``x += Z y``.  Arnoldi orthogonalization is modified
Gram-Schmidt (textbook) or classical Gram-Schmidt applied twice (Giraud,
Langou & Rozloznik, Numer. Math. 101 (2005)); the small least-squares
problem is reduced with Givens rotations.

Stopping: the recurrence residual ``|g_{j+1}| <= rtol |b|`` ends a cycle;
the true residual ``|b - J x|`` is then recomputed and the solve restarts
from ``x`` if it is still above ``rtol |b|``.  A happy breakdown is taken
when ``h_{j+1,j} <= 1e-14 |w|`` (norm before orthogonalization).
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np
import scipy.linalg as sla


@dataclass
class Info:
    iterations: int = 0
    restarts: int = 0
    converged: bool = False
    true_rel_residual: float = np.nan
    est_history: List[float] = field(default_factory=list)
    true_history: List[float] = field(default_factory=list)
    arnoldi: dict = field(default_factory=dict)


def fgmres(matvec, prec, b, x0=None, rtol=1e-8, restart=50, maxit=1000,
           ortho="mgs", keep_arnoldi=False):
    b = np.asarray(b, np.float64)
    info = Info()
    bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.float64)
    if bnorm == 0.0:
        info.converged, info.true_rel_residual = True, 0.0
        return np.zeros_like(b), info
    tol = rtol * bnorm
    while True:
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        info.true_history.append(beta / bnorm)
        info.true_rel_residual = beta / bnorm
        if beta <= tol:
            info.converged = True
            return x, info
        if info.iterations >= maxit:
            return x, info
        m = restart
        V = np.zeros((m + 1, b.size))
        Z = np.zeros((m, b.size))
        Hh = np.zeros((m + 1, m))
        Hraw = np.zeros((m + 1, m)) if keep_arnoldi else None
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = prec(V[j])
            w = matvec(Z[j])
            info.iterations += 1
            wnorm0 = float(np.linalg.norm(w))
            if ortho == "mgs":
                for i in range(j + 1):
                    Hh[i, j] = float(V[i] @ w)
                    w = w - Hh[i, j] * V[i]
            elif ortho == "cgs2":
                for _ in range(2):
                    h = V[:j + 1] @ w
                    w = w - V[:j + 1].T @ h
                    Hh[:j + 1, j] += h
            else:
                raise ValueError(ortho)
            hn = float(np.linalg.norm(w))
            Hh[j + 1, j] = hn
            breakdown = hn <= 1e-14 * wnorm0
            if not breakdown:
                V[j + 1] = w / hn
            if keep_arnoldi:
                Hraw[:, j] = Hh[:, j]
                info.arnoldi = dict(V=V[:j + 2].copy(), Z=Z[:j + 1].copy(),
                                    H=Hraw[:j + 2, :j + 1].copy())
            # Givens rotations on the new column
            col = Hh[:, j].copy()
            for i in range(j):
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1]
                col[i] = t
            rho = float(np.hypot(col[j], col[j + 1]))
            cs[j], sn[j] = col[j] / rho, col[j + 1] / rho
            col[j], col[j + 1] = rho, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            Hh[:, j] = col
            k = j + 1
            info.est_history.append(abs(g[j + 1]) / bnorm)
            if (abs(g[j + 1]) <= tol or breakdown
                    or info.iterations >= maxit):
                break
        y = sla.solve_triangular(Hh[:k, :k], g[:k], lower=False)
        x = x + Z[:k].T @ y
        info.restarts += 1
