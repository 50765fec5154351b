"""Run-to-run reproducibility.  With the apply layouts chosen by row length
(option tune = 0, the default) nothing on the path depends on timing, and
every sum has a fixed order (two-pass dot products, ordered row sums,
Galerkin products added in entry order), so two setups of one system must
give the same hierarchy, preconditioner applications, solutions and batched
solutions, bit for bit; with tune = 1 (layouts timed at setup) the sums of a
product may run in another order and are held to rounding only."""
import numpy as np
import pytest

from fracgen.configs import make_config, rhs_batch

pytestmark = pytest.mark.gpu

MC = 60


@pytest.fixture(scope="module")
def c1():
    return make_config("c1")


def _levels_bitwise(a, b):
    assert a.num_levels() == b.num_levels() >= 3
    for l in range(a.num_levels()):
        da, db = a.level_info(l), b.level_info(l)
        assert da == db, l
        for which in ((0, 1, 2) if l < a.num_levels() - 1 else (0,)):
            for ua, ub in zip(a.export_level_matrix(l, which),
                              b.export_level_matrix(l, which)):
                assert np.array_equal(ua, ub), (l, which)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_two_setups_bitwise(torch, c1, precision):
    from paper_2112_12397_amd import solver_from_system
    a = solver_from_system(c1, precision=precision, amg={"max_coarse": MC})
    b = solver_from_system(c1, precision=precision, tune=0,
                           amg={"max_coarse": MC})
    _levels_bitwise(a, b)
    for l in range(a.num_levels() - 1):
        d = a.level_info(l)
        assert all(t == 0.0 for t in d["tune_us"])
        assert all(c in (1, 4, 16, 64, 256) for c in d["layout"])
    w = torch.tensor(np.random.default_rng(11).standard_normal(c1.N),
                     device="cuda")
    va = a.apply_prec(w).clone()
    assert torch.equal(va, b.apply_prec(w))
    assert torch.equal(va, a.apply_prec(w))
    bd = torch.tensor(c1.b, device="cuda")
    xa, ia = a.solve(bd)
    xb, ib = b.solve(bd)
    assert ia["converged"] and ia["iterations"] == ib["iterations"]
    assert ia["true_rel_residual"] == ib["true_rel_residual"]
    assert torch.equal(xa, xb)
    B = torch.tensor(np.ascontiguousarray(rhs_batch(c1, 5).T), device="cuda")
    Xa, infa, _ = a.solve_batch(B)
    Xb, infb, _ = b.solve_batch(B)
    assert [i["iterations"] for i in infa] == [i["iterations"] for i in infb]
    assert torch.equal(Xa, Xb)


def test_tuned_layouts_agree_to_rounding(torch, c1):
    from paper_2112_12397_amd import solver_from_system
    a = solver_from_system(c1, tune=0, amg={"max_coarse": MC})
    t = solver_from_system(c1, tune=1, amg={"max_coarse": MC})
    w = torch.tensor(np.random.default_rng(12).standard_normal(c1.N),
                     device="cuda")
    va, vt = a.apply_prec(w), t.apply_prec(w)
    assert float(torch.linalg.norm(va - vt) / torch.linalg.norm(vt)) <= 1e-12
    bd = torch.tensor(c1.b, device="cuda")
    (xa, ia), (xt, it) = a.solve(bd), t.solve(bd)
    assert abs(ia["iterations"] - it["iterations"]) <= 1
    assert ia["converged"] and it["converged"]
    assert max(ia["true_rel_residual"], it["true_rel_residual"]) <= 1e-8
