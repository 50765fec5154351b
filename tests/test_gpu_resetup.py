"""Numeric re-setup (fpc_update_values) for the next Newton / active-set
iteration: the mesh and the first block row stay, the contact states change
C2, H (and Q2 once faces open) in values and pattern (Sec. 2.2).  The result
must equal a fresh fpc_setup on the new system, and match the oracle."""
import numpy as np
import pytest

import oracle
from fracgen import Fracture
from fracgen.configs import tiny_system

pytestmark = pytest.mark.gpu

SHAPE = (6, 6, 6)
FRS = [Fracture(0, 3, 0, 6, 0, 6), Fracture(1, 2, 0, 6, 0, 6)]
MC = 60


def _sys(slip_p=0.0, open_p=0.0, seed=7):
    return tiny_system(SHAPE, FRS, slip_p=slip_p, open_p=open_p, seed=seed)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _levels_equal(a, b):
    assert a.num_levels() == b.num_levels()
    for l in range(a.num_levels()):
        da, db = a.level_info(l), b.level_info(l)
        assert da["n_nodes"] == db["n_nodes"] and da["nnzb"] == db["nnzb"]
        assert da["lam_hi"] == db["lam_hi"]
        for which in ((0, 1, 2) if l < a.num_levels() - 1 else (0,)):
            ra, ca, va = a.export_level_matrix(l, which)
            rb, cb, vb = b.export_level_matrix(l, which)
            assert np.array_equal(ra, rb) and np.array_equal(ca, cb)
            assert np.array_equal(va, vb), (l, which)
        if l < a.num_levels() - 1:
            ga, ka = a.export_aggregates(l)
            gb, kb = b.export_aggregates(l)
            assert np.array_equal(ga, gb) and np.array_equal(ka, kb)


@pytest.mark.parametrize("mode", ["tup", "tpu"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_state_change_reuses_hierarchy(torch, mode, precision):
    """Stick -> 40% slip on the same mesh and values: the scalar patterns of
    C2 and H change, the 3x3 block pattern of S1 does not, so the AMG
    patterns are reused; hierarchy, application and solve equal a fresh
    setup on the new system and the oracle's."""
    from paper_2112_12397_amd import solver_from_system
    s0, s1 = _sys(0.0), _sys(0.4)
    assert s0.C2.nnz != s1.C2.nnz or (s0.C2 != s1.C2).nnz
    assert (s0.A != s1.A).nnz == 0
    sol = solver_from_system(s0, mode=mode, precision=precision,
                             amg={"max_coarse": MC})
    sol.update_values(s1.blocks())
    assert sol.hierarchy_reused()
    fresh = solver_from_system(s1, mode=mode, precision=precision,
                               amg={"max_coarse": MC})
    assert not fresh.hierarchy_reused()
    _levels_equal(sol, fresh)
    pc = oracle.BlockPrecond(s1.blocks(), s1.n_u, s1.n_t, s1.n_p, mode=mode,
                             coords=s1.coords,
                             amg_opts=oracle.AMGOptions(max_coarse=MC))
    rng = np.random.default_rng(3)
    w = rng.standard_normal(s1.N)
    wd = torch.tensor(w, device="cuda")
    v = sol.apply_prec(wd).cpu().numpy()
    # the same hierarchy in the same apply layouts (chosen by row length):
    # the same sums in the same order
    assert np.array_equal(v, fresh.apply_prec(wd).cpu().numpy())
    # FP32 hierarchy: the same 1e-4 bound as the FP32 parity test
    assert _rel(v, pc.apply(w)) <= (1e-10 if precision == "fp64" else 1e-4)
    x, info = sol.solve(torch.tensor(s1.b, device="cuda"))
    assert info["converged"] and info["true_rel_residual"] <= 1e-8


def test_values_change_and_second_update(torch):
    """New moduli, transmissibilities and states (another seed, same mesh),
    then back to the first system: both updates reuse the hierarchy and
    match fresh setups."""
    from paper_2112_12397_amd import solver_from_system
    sa, sb = _sys(0.3, seed=7), _sys(0.3, seed=8)
    assert (sa.A != sb.A).nnz > 0
    sol = solver_from_system(sa, amg={"max_coarse": MC})
    ref_a = solver_from_system(sa, amg={"max_coarse": MC})
    w = torch.tensor(np.random.default_rng(4).standard_normal(sa.N),
                     device="cuda")
    va = ref_a.apply_prec(w).cpu().numpy()
    sol.update_values(sb.blocks())
    assert sol.hierarchy_reused()
    _levels_equal(sol, solver_from_system(sb, amg={"max_coarse": MC}))
    sol.update_values(sa.blocks())
    assert sol.hierarchy_reused()
    _levels_equal(sol, ref_a)
    assert _rel(sol.apply_prec(w).cpu().numpy(), va) <= 1e-12


@pytest.mark.parametrize("mode", ["tup", "tpu"])
def test_faces_open(torch, mode):
    """Stick -> 30% open faces: Q2 appears (algebraic fixed stress in t-u-p,
    S~ = S1 - Q1 T~^-1 Q2 in t-p-u); whatever the hierarchy decision, the
    update equals a fresh setup and the oracle."""
    from paper_2112_12397_amd import solver_from_system
    s0, s1 = _sys(0.0), _sys(0.2, 0.3)
    assert s0.Q2.nnz == 0 and s1.Q2.nnz > 0
    sol = solver_from_system(s0, mode=mode, amg={"max_coarse": MC})
    sol.update_values(s1.blocks())
    fresh = solver_from_system(s1, mode=mode, amg={"max_coarse": MC})
    _levels_equal(sol, fresh)
    pc = oracle.BlockPrecond(s1.blocks(), s1.n_u, s1.n_t, s1.n_p, mode=mode,
                             coords=s1.coords,
                             amg_opts=oracle.AMGOptions(max_coarse=MC))
    w = np.random.default_rng(5).standard_normal(s1.N)
    v = sol.apply_prec(torch.tensor(w, device="cuda")).cpu().numpy()
    assert _rel(v, pc.apply(w)) <= 1e-10
    x, info = sol.solve(torch.tensor(s1.b, device="cuda"))
    assert info["converged"] and info["true_rel_residual"] <= 1e-8


def test_update_errors(torch):
    from paper_2112_12397_amd import FpcError, solver_from_system
    s0 = _sys(0.0)
    sol = solver_from_system(s0, amg={"max_coarse": MC})
    other = tiny_system((4, 4, 4), seed=1)
    with pytest.raises(FpcError) as e:
        sol.update_values(other.blocks())
    assert e.value.status == -2
    # a failed size check leaves the handle as it was
    w = torch.zeros(s0.N, dtype=torch.float64, device="cuda")
    sol.apply_prec(w)
    bad = s0.blocks()
    A = bad["A"].copy()
    A.data[3] = np.inf
    bad["A"] = A
    with pytest.raises(FpcError) as e:
        sol.update_values(bad)
    assert e.value.status == -6
    # a failed update leaves the handle not set up until the next setup
    for call in (lambda: sol.apply_prec(w),
                 lambda: sol.update_values(s0.blocks())):
        with pytest.raises(FpcError) as e:
            call()
        assert e.value.status == -9
    sol.setup(s0.blocks(), s0.coords)
    assert not sol.hierarchy_reused()
    sol.apply_prec(w)
