"""fpc_grad_log_trans_noalloc (static device work area, no allocation in the
call) against fpc_grad_log_trans (work area allocated per call), through the
C ABI: two calls in a row on one GPU, the second with a smaller input, so
the second runs on the array the first left behind.  Both entry points run
the same kernels in the same order, so the results must agree bit for bit;
each is also checked against the oracle's gradient formula."""
import numpy as np
import pytest

import fracgen
import oracle
from fracgen import tiny_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _case(torch, s, seed):
    from paper_2112_12397_amd import solver_from_system
    sol = solver_from_system(s)
    rng = np.random.default_rng(seed)
    lam = rng.standard_normal(s.n_p)
    p = rng.standard_normal(s.n_p)
    dev = lambda a: torch.tensor(a, device="cuda")  # noqa: E731
    return sol, lam, p, dev(lam), dev(p)


def _ref(s, pairs, lam, p):
    return oracle.adjoint.grad_log_trans(pairs, s.flow_ndir, s.upsilon, lam, p)


def test_noalloc_matches_allocating_entry_point(torch):
    big = fracgen.make_config("c1")                   # 100 faces
    small = tiny_system((4, 4, 4), seed=1)            # 16 faces
    assert small.n_p < big.n_p
    runs = []
    for s, seed in ((big, 3), (small, 4)):
        sol, lam, p, dlam, dp = _case(torch, s, seed)
        runs.append((s, sol, lam, p, dlam, dp))
    for s, sol, lam, p, dlam, dp in runs:
        graph, keep = sol.flow_graph(torch.tensor(s.flow_pairs),
                                     torch.tensor(s.flow_ndir),
                                     torch.tensor(s.upsilon))
        out = torch.full((s.n_p,), np.nan, dtype=torch.float64, device="cuda")
        sol.grad_log_trans_noalloc(graph, dlam, dp, out)
        got = out.cpu().numpy()
        want = sol.grad_log_trans(torch.tensor(s.flow_pairs),
                                  torch.tensor(s.flow_ndir),
                                  torch.tensor(s.upsilon), dlam, dp)
        assert np.array_equal(got, want.cpu().numpy())
        ref = _ref(s, s.flow_pairs, lam, p)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
        del keep
    # the same handle again with fewer pairs (a smaller work area than the
    # previous call left in the array)
    s, sol, lam, p, dlam, dp = runs[0]
    sub = s.flow_pairs[::3].copy()
    graph, keep = sol.flow_graph(torch.tensor(sub), torch.tensor(s.flow_ndir),
                                 torch.tensor(s.upsilon))
    out = torch.empty(s.n_p, dtype=torch.float64, device="cuda")
    got = sol.grad_log_trans_noalloc(graph, dlam, dp, out).cpu().numpy()
    want = sol.grad_log_trans(torch.tensor(sub), torch.tensor(s.flow_ndir),
                              torch.tensor(s.upsilon), dlam, dp)
    assert np.array_equal(got, want.cpu().numpy())
    ref = _ref(s, sub, lam, p)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_noalloc_rejects_oversized_and_bad_input(torch):
    from paper_2112_12397_amd.fracprec import FpcError
    s = tiny_system((4, 4, 4), seed=1)
    sol, lam, p, dlam, dp = _case(torch, s, 5)
    nd, up = torch.tensor(s.flow_ndir), torch.tensor(s.upsilon)
    # 2 n_p + 1 + 2 n_pairs > 2^20 words: refused before any kernel runs
    m = (1 << 19) + 1
    pairs = torch.tensor(np.tile(s.flow_pairs[:1], (m, 1)))
    graph, keep = sol.flow_graph(pairs, nd, up)
    out = torch.full((s.n_p,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(FpcError, match="FPC_ERR_ARG.*static maximum"):
        sol.grad_log_trans_noalloc(graph, dlam, dp, out)
    assert torch.all(out == 7.0)
    del keep
    # an invalid pair is caught by the validation pass, output untouched
    bad = np.vstack([s.flow_pairs, [[0, s.n_p]]])
    graph, keep = sol.flow_graph(torch.tensor(bad), nd, up)
    with pytest.raises(FpcError, match="FPC_ERR_PATTERN"):
        sol.grad_log_trans_noalloc(graph, dlam, dp, out)
    assert torch.all(out == 7.0)
    del keep
    # and a valid call right after the refused ones
    graph, keep = sol.flow_graph(torch.tensor(s.flow_pairs), nd, up)
    got = sol.grad_log_trans_noalloc(graph, dlam, dp, out).cpu().numpy()
    ref = _ref(s, s.flow_pairs, lam, p)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
