"""Pins of the oracle's adjoint gradients."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from fracgen import Fracture, tiny_system, assemble_T
from oracle.adjoint import fd_grad_log_trans, grad_log_trans, loss_and_grad_x


def _sys():
    return tiny_system((5, 5, 5), [Fracture(0, 2, 0, 5, 0, 5),
                                   Fracture(1, 3, 1, 4, 1, 4)], seed=7)


def _pc(s):
    return oracle.BlockPrecond(s.blocks(), s.n_u, s.n_t, s.n_p,
                               coords=s.coords,
                               amg_opts=oracle.AMGOptions(max_coarse=60))


def test_adjoint_structure():
    """Q2 = 0: lambda_u = lambda_t = 0 and lambda_p = T^{-T} g_p."""
    s = _sys()
    pc = _pc(s)
    rng = np.random.default_rng(0)
    g = np.zeros(s.N)
    g[s.n_u + s.n_t:] = rng.standard_normal(s.n_p)
    lam, info = oracle.fgmres(pc.matvec_T, pc.apply_T, g, rtol=1e-12)
    assert info.converged
    lp = spla.spsolve(sp.csc_matrix(s.T.T), g[s.n_u + s.n_t:])
    assert np.linalg.norm(lam[s.n_u + s.n_t:] - lp) <= 1e-9 * np.linalg.norm(lp)
    assert np.abs(lam[:s.n_u + s.n_t]).max() <= 1e-9 * np.abs(lp).max()
    # linearity in the right-hand side
    lam2, _ = oracle.fgmres(pc.matvec_T, pc.apply_T, 3.0 * g, rtol=1e-12)
    assert np.allclose(lam2, 3.0 * lam, rtol=1e-8, atol=1e-8 * np.abs(lam).max())


def test_gradient_matches_extended_precision_fd():
    s = _sys()
    pc = _pc(s)
    rng = np.random.default_rng(1)
    p_obs = rng.standard_normal(s.n_p) * 1e3
    x, info = oracle.fgmres(pc.matvec, pc.apply, s.b, rtol=1e-12)
    L, g = loss_and_grad_x(x, s.n_u, s.n_t, p_obs)
    lam, _ = oracle.fgmres(pc.matvec_T, pc.apply_T, g, rtol=1e-12)
    p = x[s.n_u + s.n_t:]
    grad = grad_log_trans(s.flow_pairs, s.flow_ndir, s.upsilon,
                          lam[s.n_u + s.n_t:], p)
    faces = rng.choice(s.n_p, 8, replace=False)
    fd = fd_grad_log_trans(s.flow_pairs, s.flow_ndir, s.upsilon, s.T_stab,
                           s.b[s.n_u + s.n_t:], p_obs, faces)
    scale = np.abs(fd).max()
    assert np.abs(grad[faces] - fd).max() <= 1e-6 * scale
    # the generator's T(U) is the matrix the gradient differentiates
    assert abs(assemble_T(s, s.upsilon) - s.T).max() == 0
