"""Extra synthetic systems for the GPU tests (test infrastructure)."""
import numpy as np
import scipy.sparse as sp

from fracgen import tiny_system


def wide_system():
    """A tiny system whose A gains graph-Laplacian couplings (times I3)
    between four hub nodes next to the fracture and 300 other nodes each:
    block rows longer than the one-wavefront and LDS limits of the setup
    kernels (CSR to 3x3 blocks, S1 = A + C1 H~^-1 C2, sliced-ELL fill)."""
    import dataclasses
    s = tiny_system((8, 8, 8), slip_p=0.3, seed=7)
    rng = np.random.default_rng(11)
    nn = s.n_u // 3
    free = ~s.dirichlet.reshape(nn, 3).any(axis=1)
    frac_nodes = np.unique(s.C1.tocoo().row // 3)
    hubs = [h for h in frac_nodes if free[h]][:4]
    cand = np.flatnonzero(free)
    eps = 1e-3 * s.A.diagonal().mean()
    rows, cols, vals = [], [], []
    for h in hubs:
        for j in rng.choice(cand[cand != h], size=300, replace=False):
            for d in range(3):
                a, b = 3 * h + d, 3 * j + d
                rows += [a, b, a, b]
                cols += [a, b, b, a]
                vals += [eps, eps, -eps, -eps]
    A = (s.A + sp.csr_matrix((vals, (rows, cols)), shape=s.A.shape)).tocsr()
    A.sort_indices()
    return dataclasses.replace(s, A=A)
