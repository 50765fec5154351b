"""Production forms on the GPU: batched right-hand sides, the FP32
preconditioner and the adjoint / autograd gradients (full 48^3 workload)."""
import numpy as np
import pytest

import fracgen
import oracle
from fracgen.configs import observations, rhs_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def c1():
    return fracgen.make_config("c1")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


_PC = {}


def _c1_oracle(s):
    if "c1" not in _PC:
        _PC["c1"] = oracle.BlockPrecond(s.blocks(), s.n_u, s.n_t, s.n_p,
                                        coords=s.coords)
    return _PC["c1"]


@pytest.mark.parametrize("k", [3, 12])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_matches_oracle_and_single(torch, c1, k, precision):
    """Every column of a batched solve (norms 1e-2 .. 1e2) against the FP64
    oracle's FGMRES(50) with CGS2 on that column: iterations within 2 of the
    oracle's, solution within 1e-5 relative (both precisions of the
    hierarchy; the observed errors are printed), true residual <= 1e-8
    recomputed on the host; and against the GPU's own single solve."""
    from paper_2112_12397_amd import solver_from_system
    s = c1
    pc = _c1_oracle(s)
    sol = solver_from_system(s, precision=precision)
    B = rhs_batch(s, k=k)                      # norms 1e-2 .. 1e2
    Bt = torch.tensor(np.ascontiguousarray(B.T), device="cuda")
    X, infos, status = sol.solve_batch(Bt)
    assert status == "FPC_OK"
    J = s.jacobian()
    Xn = X.cpu().numpy()
    errs = []
    for c in range(k):
        xo, io = oracle.fgmres(pc.matvec, pc.apply, B[:, c], rtol=1e-8,
                               ortho="cgs2")
        x1, i1 = sol.solve(Bt[c].contiguous())
        r = np.linalg.norm(B[:, c] - J @ Xn[c]) / np.linalg.norm(B[:, c])
        assert infos[c]["converged"] == 1 and r <= 1e-8, (c, r, infos[c])
        assert abs(infos[c]["iterations"] - io.iterations) <= 2, \
            (c, infos[c]["iterations"], io.iterations)
        errs.append(_rel(Xn[c], xo))
        assert errs[-1] <= 1e-5, (c, errs[-1])
        assert abs(infos[c]["iterations"] - i1["iterations"]) <= 2
        assert _rel(Xn[c], x1.cpu().numpy()) <= 1e-5
    print(f"batch {precision} k={k}: max |x - x_oracle| / |x_oracle| = "
          f"{max(errs):.2e}")


@pytest.mark.parametrize("k", [5])
def test_batch_short_cycles(torch, c1, k):
    """Batched FGMRES(7) with the delayed Gram-Schmidt: columns of different
    norms restart at different steps, every cycle ends with the finalizing
    pass; each column against the oracle's CGS2 FGMRES(7) (iterations
    within 2, solution within 1e-5) and its own single solve."""
    from paper_2112_12397_amd import solver_from_system
    s = c1
    pc = _c1_oracle(s)
    sol = solver_from_system(s, restart=7)
    B = rhs_batch(s, k=k)
    Bt = torch.tensor(np.ascontiguousarray(B.T), device="cuda")
    X, infos, status = sol.solve_batch(Bt)
    assert status == "FPC_OK"
    J = s.jacobian()
    Xn = X.cpu().numpy()
    for c in range(k):
        xo, io = oracle.fgmres(pc.matvec, pc.apply, B[:, c], rtol=1e-8,
                               restart=7, ortho="cgs2")
        x1, i1 = sol.solve(Bt[c].contiguous())
        r = np.linalg.norm(B[:, c] - J @ Xn[c]) / np.linalg.norm(B[:, c])
        assert infos[c]["converged"] == 1 and r <= 1e-8, (c, r, infos[c])
        assert infos[c]["restarts"] > 2
        assert abs(infos[c]["iterations"] - io.iterations) <= 2, \
            (c, infos[c]["iterations"], io.iterations)
        assert abs(infos[c]["iterations"] - i1["iterations"]) <= 2
        assert _rel(Xn[c], xo) <= 1e-5
        assert _rel(Xn[c], x1.cpu().numpy()) <= 1e-5


@pytest.mark.parametrize("ortho", ["dcgs2", "cgs2"])
def test_batch_long_cycle(torch, ortho):
    """Batched FGMRES(63) to 1e-9 on the long-row system with random
    right-hand sides: the oracle needs 56-57 steps in one cycle, so the
    batched Gram-Schmidt passes go past 48 basis vectors per column (CGS2:
    the axpy and dot passes run separately there; delayed: the dot pass in
    two launches past 32, the finalizing pass over 57 vectors); every column
    against the oracle (CGS2) and its single solve.  (Closer to this
    system's attainable accuracy, about 5e-12, counts become
    rounding-sensitive: at 1e-10 the oracle's CGS2 and MGS counts already
    differ by up to 5.)"""
    from paper_2112_12397_amd import solver_from_system
    from systems_extra import wide_system
    s = wide_system()
    sol = solver_from_system(s, restart=63, ortho=ortho,
                             amg={"max_coarse": 90})
    pc = oracle.BlockPrecond(s.blocks(), s.n_u, s.n_t, s.n_p, coords=s.coords,
                             amg_opts=oracle.AMGOptions(max_coarse=90))
    rng = np.random.default_rng(21)
    B = rng.standard_normal((s.N, 4)) * np.array([1e-2, 1.0, 1e2, 3.0])
    Bt = torch.tensor(np.ascontiguousarray(B.T), device="cuda")
    X, infos, status = sol.solve_batch(Bt, rtol=1e-9)
    assert status == "FPC_OK"
    J = s.jacobian()
    Xn = X.cpu().numpy()
    for c in range(4):
        xo, io = oracle.fgmres(pc.matvec, pc.apply, B[:, c], rtol=1e-9,
                               restart=63, ortho="cgs2")
        x1, i1 = sol.solve(Bt[c].contiguous(), rtol=1e-9)
        r = np.linalg.norm(B[:, c] - J @ Xn[c]) / np.linalg.norm(B[:, c])
        assert infos[c]["converged"] == 1 and r <= 1e-9, (c, r, infos[c])
        assert i1["iterations"] > 48            # past 48 basis vectors
        assert abs(infos[c]["iterations"] - io.iterations) <= 2
        assert abs(infos[c]["iterations"] - i1["iterations"]) <= 2
        assert _rel(Xn[c], xo) <= 1e-6
        assert _rel(Xn[c], x1.cpu().numpy()) <= 1e-6


def test_batch_zero_column_and_mask(torch, c1):
    from paper_2112_12397_amd import solver_from_system
    s = c1
    sol = solver_from_system(s)
    B = rhs_batch(s, k=4)
    B[:, 2] = 0.0                              # a zero column converges at once
    Bt = torch.tensor(np.ascontiguousarray(B.T), device="cuda")
    X, infos, status = sol.solve_batch(Bt)
    assert status == "FPC_OK"
    assert infos[2]["iterations"] == 0 and not X[2].any()
    for c in (0, 1, 3):
        assert infos[c]["converged"] == 1 and infos[c]["iterations"] > 0


def test_adjoint_gradients_c5(torch):
    """48^3 with 4 full fractures: gradients of 0.5 |p - p_obs|^2 with respect
    to log transmissibility on 20 seeded faces against central differences
    (h = 1e-6, 80-bit) and against the oracle's adjoint gradient; the
    gradient with respect to b is the adjoint solution.  The forward solve
    to 1e-8 also matches the oracle's FGMRES (iterations within 2, solution
    within 1e-5)."""
    from paper_2112_12397_amd import solver_from_system
    from paper_2112_12397_amd.autograd import SolveFn
    s = fracgen.make_config("c5")
    _, p_obs = observations(s)
    sol = solver_from_system(s)
    off = s.n_u + s.n_t
    b = torch.tensor(s.b, device="cuda", requires_grad=True)
    logu = torch.tensor(np.log(s.upsilon), device="cuda", requires_grad=True)
    flow = (torch.tensor(s.flow_pairs), torch.tensor(s.flow_ndir))
    x = SolveFn.apply(b, logu, sol, flow, 1e-11)
    pobs = torch.tensor(p_obs, device="cuda")
    loss = 0.5 * ((x[off:] - pobs) ** 2).sum()
    loss.backward()
    g_logu = logu.grad.cpu().numpy()
    g_b = b.grad.cpu().numpy()
    rng = np.random.default_rng(2024)
    faces = rng.choice(s.n_p, 20, replace=False)
    fd = oracle.adjoint.fd_grad_log_trans(s.flow_pairs, s.flow_ndir,
                                          s.upsilon, s.T_stab, s.b[off:],
                                          p_obs, faces, h=1e-6)
    err = np.abs(g_logu[faces] - fd)
    assert (err <= 1e-6 * np.abs(fd) + 1e-9 * np.abs(fd).max()).all(), \
        (err / np.abs(fd)).max()
    # oracle adjoint (its own forward and adjoint FGMRES)
    pc = oracle.BlockPrecond(s.blocks(), s.n_u, s.n_t, s.n_p, coords=s.coords)
    # the forward solve at the workload tolerance against the oracle's
    x8, i8 = sol.solve(torch.tensor(s.b, device="cuda"))
    xo8, io8 = oracle.fgmres(pc.matvec, pc.apply, s.b, rtol=1e-8, ortho="cgs2")
    print(f"c5: GPU {i8['iterations']} iterations, oracle {io8.iterations}")
    assert abs(i8["iterations"] - io8.iterations) <= 2
    assert _rel(x8.cpu().numpy(), xo8) <= 1e-5
    xo, _ = oracle.fgmres(pc.matvec, pc.apply, s.b, rtol=1e-11)
    L, gx = oracle.adjoint.loss_and_grad_x(xo, s.n_u, s.n_t, p_obs)
    lam, _ = oracle.fgmres(pc.matvec_T, pc.apply_T, gx, rtol=1e-11)
    go = oracle.adjoint.grad_log_trans(s.flow_pairs, s.flow_ndir, s.upsilon,
                                       lam[off:], xo[off:])
    assert _rel(g_logu, go) <= 1e-7
    assert _rel(g_b, lam) <= 1e-7
    # with no open faces the adjoint has zero displacement / traction parts
    assert np.abs(g_b[:off]).max() <= 1e-8 * np.abs(g_b[off:]).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_graph_replays_match_eager(torch, c1, precision):
    """The batched V-cycle replayed from its captured HIP graph gives the
    eager result bit for bit, on every replay, with eager single-column
    solves and synchronisations between the replays."""
    from paper_2112_12397_amd import solver_from_system
    s = c1
    B = rhs_batch(s, k=5)
    Bt = torch.tensor(np.ascontiguousarray(B.T), device="cuda")
    eager = solver_from_system(s, precision=precision, graphs=0)
    X0, i0, st0 = eager.solve_batch(Bt)
    assert st0 == "FPC_OK"
    graph = solver_from_system(s, precision=precision)   # graphs on
    for rep in range(3):
        Xg, ig, stg = graph.solve_batch(Bt)
        torch.cuda.synchronize()
        assert stg == "FPC_OK"
        assert torch.equal(Xg, X0), rep
        assert [d["iterations"] for d in ig] == [d["iterations"] for d in i0]
        x1, inf1 = graph.solve(Bt[rep].contiguous())
        torch.cuda.synchronize()
        assert inf1["converged"] == 1


def test_batch_full_size_c4(torch):
    """64^3 mesh with 6 random fractures: 32 right-hand sides (norms 1e-2 ..
    1e2) in one batch, FP32 preconditioner, FP64 outer solve; every column
    reaches a true relative residual <= 1e-8, recomputed on the host."""
    from paper_2112_12397_amd import solver_from_system
    s = fracgen.make_config("c4")
    sol = solver_from_system(s, precision="fp32")
    B = rhs_batch(s, k=32)
    Bt = torch.tensor(np.ascontiguousarray(B.T), device="cuda")
    X, infos, status = sol.solve_batch(Bt)
    assert status == "FPC_OK"
    J = s.jacobian()
    Xn = X.cpu().numpy()
    for c in range(32):
        r = np.linalg.norm(B[:, c] - J @ Xn[c]) / np.linalg.norm(B[:, c])
        assert infos[c]["converged"] == 1 and r <= 1e-8, (c, r, infos[c])
