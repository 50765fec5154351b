"""Pins of the oracle's FGMRES against dense linear algebra."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import fracgen
from fracgen import Fracture, tiny_system
from oracle.amg import AMGOptions


def _pc(s, inner="amg"):
    return oracle.BlockPrecond(s.blocks(), s.n_u, s.n_t, s.n_p, coords=s.coords,
                               inner=inner, amg_opts=AMGOptions(max_coarse=40))


@pytest.mark.parametrize("ortho", ["mgs", "cgs2"])
def test_matches_dense_lu(ortho):
    s = tiny_system((4, 4, 4), slip_p=0.3, seed=2)
    pc = _pc(s)
    J = s.jacobian().toarray()
    xd = np.linalg.solve(J, s.b)
    x, info = oracle.fgmres(pc.matvec, pc.apply, s.b, rtol=1e-10,
                            restart=30, ortho=ortho)
    assert info.converged and info.true_rel_residual <= 1e-10
    kappa = np.linalg.cond(J)
    assert np.linalg.norm(x - xd) <= kappa * 1e-10 * np.linalg.norm(xd)
    est = np.array(info.est_history)
    assert (np.diff(est) <= 1e-14).all()           # monotone estimate


def test_arnoldi_relation():
    s = tiny_system((3, 3, 3), seed=1)
    pc = _pc(s)
    x, info = oracle.fgmres(pc.matvec, pc.apply, s.b, rtol=1e-12,
                            restart=8, maxit=8, keep_arnoldi=True)
    V, Z, H = (info.arnoldi[k] for k in ("V", "Z", "H"))
    k = Z.shape[0]
    JZ = np.stack([pc.matvec(z) for z in Z], axis=1)
    assert np.abs(JZ - V.T @ H).max() <= 1e-12 * np.abs(JZ).max()
    assert np.abs(V @ V.T - np.eye(k + 1)).max() < 1e-12


def test_identity_preconditioner_and_breakdown():
    rng = np.random.default_rng(0)
    n = 12
    A = rng.standard_normal((n, n)) + n * np.eye(n)
    b = rng.standard_normal(n)
    x, info = oracle.fgmres(lambda v: A @ v, lambda v: v, b, rtol=1e-12,
                            restart=n)
    assert info.iterations <= n and info.converged
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10)
    # happy breakdown: the identity operator is solved in one step
    x, info = oracle.fgmres(lambda v: v, lambda v: v, b, rtol=1e-12)
    assert info.iterations == 1 and np.allclose(x, b)
    # zero right-hand side
    x, info = oracle.fgmres(lambda v: A @ v, lambda v: v, np.zeros(n))
    assert info.iterations == 0 and not x.any()


def test_restart_and_maxit():
    s = tiny_system((4, 4, 4), seed=4)
    pc = _pc(s)
    x, info = oracle.fgmres(pc.matvec, pc.apply, s.b, rtol=1e-10, restart=12)
    assert info.converged and info.restarts > 1
    x2, info2 = oracle.fgmres(pc.matvec, pc.apply, s.b, rtol=1e-10, maxit=2)
    assert not info2.converged and info2.iterations == 2


def test_c1_solution_matches_sparse_direct():
    s = fracgen.make_config("c1")
    pc = oracle.BlockPrecond(s.blocks(), s.n_u, s.n_t, s.n_p, coords=s.coords)
    x, info = oracle.fgmres(pc.matvec, pc.apply, s.b, rtol=1e-8)
    assert info.converged and info.true_rel_residual <= 1e-8
    xd = spla.spsolve(s.jacobian().tocsc(), s.b)
    assert np.linalg.norm(x - xd) <= 1e-5 * np.linalg.norm(xd)
    assert 10 <= info.iterations <= 60
