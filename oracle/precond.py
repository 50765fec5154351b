"""Block preconditioners M1 (t-p-u) and M2 (t-u-p), step by step.

* construction ``cpt_tpu`` / ``cpt_tup``: Alg 3.1 / Alg 3.3,
* application ``app_tpu`` / ``app_tup``: Alg 3.2 / Alg 3.4,
* transposed applications ``M^{-T}``: the factors of eq. P1 / eq. P2
  transposed and applied in reverse order (used by the adjoint solve).

The inner operator on the mechanics block is either the AMG V-cycle or, for
exactness checks, a sparse direct solve.  The pressure-block solves use a
sparse direct factorization (the paper's nested direct solver).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .amg import AMGOptions, build_hierarchy
from .blocks import (bdiag_apply, bdiag_inv, fixed_stress, node_pattern,
                     bool_product, s1_node_pattern, schur1, schur_tpu)


class BlockPrecond:
    def __init__(self, blocks, n_u, n_t, n_p, mode="tup", inner="amg",
                 coords=None, amg_opts=None):
        if mode not in ("tup", "tpu", "tup_star"):
            raise ValueError(mode)
        self.mode, self.inner_kind = mode, inner
        self.n_u, self.n_t, self.n_p = n_u, n_t, n_p
        b = {k: sp.csr_matrix(v) for k, v in blocks.items()}
        self.A, self.C1, self.Q1 = b["A"], b["C1"], b["Q1"]
        self.C2, self.H, self.Q2, self.T = b["C2"], b["H"], b["Q2"], b["T"]
        self.C1T = sp.csr_matrix(self.C1.T)
        self.C2T = sp.csr_matrix(self.C2.T)
        self.Q1T = sp.csr_matrix(self.Q1.T)
        self.Q2T = sp.csr_matrix(self.Q2.T)
        # H~ = Bdiag(H, 3)
        self.Hinv = bdiag_inv(self.H, n_p)
        pattern = s1_node_pattern(self.A, self.C1, self.C2)
        if mode in ("tup", "tup_star"):
            # Alg 3.3: S1 = A + C1 H~^{-1} C2;  S~2 = T - FS(Q2, S1, Q1)
            self.K = schur1(self.A, self.C1, self.Hinv, self.C2)
            self.S_K = fixed_stress(self.K, self.Q1, self.Q2)
            self.S2t = sp.csr_matrix(self.T - sp.diags(self.S_K))
            self.p_lu = spla.splu(sp.csc_matrix(self.S2t))
        else:
            # Alg 3.1: S~ = A + C1 H~^{-1} C2 - Q1 T~^{-1} Q2, T~ = diag(T)
            self.K = schur_tpu(self.A, self.C1, self.Hinv, self.C2, self.Q1,
                               self.T, self.Q2)
            if self.Q2.nnz:
                pattern = sp.csr_matrix(
                    pattern.astype(np.int64) + bool_product(
                        node_pattern(self.Q1, 3, 1),
                        node_pattern(self.Q2, 1, 3)).astype(np.int64))
                pattern.data[:] = 1
                pattern = pattern.astype(np.int8)
            self.p_lu = spla.splu(sp.csc_matrix(self.T))
        self.pattern = pattern
        if inner == "amg":
            self.amg = build_hierarchy(self.K, pattern, coords,
                                       amg_opts or AMGOptions())
        elif inner == "exact":
            self.K_lu = spla.splu(sp.csc_matrix(self.K))
        else:
            raise ValueError(inner)

    # -- inner operators ----------------------------------------------------
    def inner(self, y, transpose=False):
        """AMG(K, y) (or the exact K^{-1} y)."""
        if self.inner_kind == "amg":
            return self.amg.vcycle(y, transpose=transpose)
        return self.K_lu.solve(y, trans="T" if transpose else "N")

    def psolve(self, y, transpose=False):
        return self.p_lu.solve(y, trans="T" if transpose else "N")

    def split(self, w):
        nu, nt = self.n_u, self.n_t
        return w[:nu], w[nu:nu + nt], w[nu + nt:]

    # -- applications -------------------------------------------------------
    def apply(self, w):
        """v = M^{-1} w."""
        return {"tup": self._tup, "tpu": self._tpu,
                "tup_star": self._tup_star}[self.mode](w)

    def apply_T(self, w):
        """v = M^{-T} w."""
        return {"tup": self._tup_T, "tpu": self._tpu_T,
                "tup_star": self._tup_star_T}[self.mode](w)

    def _tup(self, w):
        """Alg 3.4 (app_tup)."""
        w_u, w_t, w_p = self.split(np.asarray(w, np.float64))
        t_t = bdiag_apply(self.Hinv, w_t)
        t_u = w_u + self.C1 @ t_t
        s_u = self.inner(t_u)
        t_p = w_p - self.Q2 @ s_u
        v_p = self.psolve(t_p)
        t_u = self.Q1 @ v_p
        v_u = self.inner(t_u)
        v_u = s_u - v_u
        s_t = self.C2 @ v_u
        v_t = -t_t + bdiag_apply(self.Hinv, s_t)
        return np.concatenate([v_u, v_t, v_p])

    def _tup_T(self, w):
        """M2^{-T} = L2^{-T} D2^{-T} U2^{-T} of eq. P2: Alg 3.4 with C1 and
        C2^T, Q1 and Q2^T exchanged and every operator transposed."""
        w_u, w_t, w_p = self.split(np.asarray(w, np.float64))
        t_t = bdiag_apply(self.Hinv, w_t, transpose=True)
        t_u = w_u + self.C2T @ t_t
        s_u = self.inner(t_u, transpose=True)
        t_p = w_p - self.Q1T @ s_u
        v_p = self.psolve(t_p, transpose=True)
        t_u = self.Q2T @ v_p
        v_u = self.inner(t_u, transpose=True)
        v_u = s_u - v_u
        s_t = self.C1T @ v_u
        v_t = -t_t + bdiag_apply(self.Hinv, s_t, transpose=True)
        return np.concatenate([v_u, v_t, v_p])

    def _tup_star(self, w):
        """M2*^{-1} = D2^{-1} L2^{-1} of eq. LDU2 (the incomplete block
        factorization of the remark after Prop 3.2), in the t-u-p order:
        steps 1-5 of Alg 3.4 with v_u = s_u and v_t = -t_t."""
        w_u, w_t, w_p = self.split(np.asarray(w, np.float64))
        t_t = bdiag_apply(self.Hinv, w_t)
        v_u = self.inner(w_u + self.C1 @ t_t)
        v_p = self.psolve(w_p - self.Q2 @ v_u)
        return np.concatenate([v_u, -t_t, v_p])

    def _tup_star_T(self, w):
        """M2*^{-T} = L2^{-T} D2^{-T}."""
        w_u, w_t, w_p = self.split(np.asarray(w, np.float64))
        v_p = self.psolve(w_p, transpose=True)
        v_u = self.inner(w_u - self.Q2T @ v_p, transpose=True)
        t_t = bdiag_apply(self.Hinv, w_t, transpose=True)
        v_t = -t_t + bdiag_apply(self.Hinv, self.C1T @ v_u, transpose=True)
        return np.concatenate([v_u, v_t, v_p])

    def _tpu(self, w):
        """Alg 3.2 (app_tpu)."""
        w_u, w_t, w_p = self.split(np.asarray(w, np.float64))
        t_p = self.psolve(w_p)
        t_t = bdiag_apply(self.Hinv, w_t)
        t_u = w_u + self.C1 @ t_t - self.Q1 @ t_p
        v_u = self.inner(t_u)
        s_p = self.Q2 @ v_u
        s_t = self.C2 @ v_u
        v_p = t_p - self.psolve(s_p)
        v_t = -t_t + bdiag_apply(self.Hinv, s_t)
        return np.concatenate([v_u, v_t, v_p])

    def _tpu_T(self, w):
        """M1^{-T} = L1^T D1^{-T} U1^T of eq. P1 (transposed factors)."""
        w_u, w_t, w_p = self.split(np.asarray(w, np.float64))
        t_p = self.psolve(w_p, transpose=True)
        t_t = bdiag_apply(self.Hinv, w_t, transpose=True)
        t_u = w_u + self.C2T @ t_t - self.Q2T @ t_p
        v_u = self.inner(t_u, transpose=True)
        s_p = self.Q1T @ v_u
        s_t = self.C1T @ v_u
        v_p = t_p - self.psolve(s_p, transpose=True)
        v_t = -t_t + bdiag_apply(self.Hinv, s_t, transpose=True)
        return np.concatenate([v_u, v_t, v_p])

    # -- the Jacobian -------------------------------------------------------
    def matvec(self, x):
        """J x with J = [A C1 Q1; C2 -H 0; Q2 0 T] (eq. JacSys)."""
        x_u, x_t, x_p = self.split(np.asarray(x, np.float64))
        return np.concatenate([self.A @ x_u + self.C1 @ x_t + self.Q1 @ x_p,
                               self.C2 @ x_u - self.H @ x_t,
                               self.Q2 @ x_u + self.T @ x_p])

    def matvec_T(self, x):
        """J^T x."""
        x_u, x_t, x_p = self.split(np.asarray(x, np.float64))
        return np.concatenate([self.A.T @ x_u + self.C2T @ x_t + self.Q2T @ x_p,
                               self.C1T @ x_u - self.H.T @ x_t,
                               self.Q1T @ x_u + self.T.T @ x_p])
