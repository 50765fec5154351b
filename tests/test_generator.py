"""Pins of the synthetic block system against what the paper fixes.

* dof counting of Table test2a (node splitting convention),
* A symmetric positive definite, C2 = C1^T in stick, H SPSD and singular,
  T SPD with the 2D stencil, no traction/pressure coupling (Sec. 2.2),
* a uniform-strain patch test of the first two block rows,
* seed determinism.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import fracgen
from fracgen import Fracture, tiny_system
from fracgen.problem import POISSON, build_system


def test_counts_c1():
    s = fracgen.make_config("c1")
    # 11^3 nodes + 121 split copies on the fully cut plane
    assert s.n_u == 3 * (11 ** 3 + 121) == 4356
    assert s.n_p == 100 and s.n_t == 300


def test_counts_table_test2a():
    """Table test2a: 25^3 and 50^3 cubes with 4 embedded fractures of
    15x15 / 30x30 faces: n_u = 55,080 / 408,045, n_t = 2,700 / 10,800,
    n_p = 900 / 3,600 (only fracture-interior nodes are split)."""
    for n, side, exp in ((25, 15, (55080, 2700, 900)),
                         (50, 30, (408045, 10800, 3600))):
        lo = (n - side) // 2
        fr = [Fracture(0, q, lo, lo + side, lo, lo + side)
              for q in np.linspace(n // 5, 4 * n // 5, 4).astype(int)]
        E = np.full(n ** 3, 1e4)
        s = build_system((n, n, n), 1.0 / n, fr, E,
                         np.full(4 * side * side, 1e-10))
        assert (s.n_u, s.n_t, s.n_p) == exp
        assert s.N == sum(exp)


def test_counts_c2_splitting():
    """Three orthogonal full planes: 1 extra copy per single-plane node,
    3 per line node, 7 at the centre (19,927 extra nodes)."""
    n = 8
    fr = [Fracture(a, n // 2, 0, n, 0, n) for a in range(3)]
    s = build_system((n, n, n), 1.0 / n, fr, np.full(n ** 3, 1e4),
                     np.full(3 * n * n, 1e-10))
    nn = n + 1
    plane_only = 3 * (nn * nn - 2 * nn + 1)
    line_only = 3 * (nn - 1)
    extra = plane_only + 3 * line_only + 7
    assert s.n_u == 3 * (nn ** 3 + extra)
    # the formula at 80^3 gives the c2 count
    nn = 81
    extra80 = 3 * (nn * nn - 2 * nn + 1) + 3 * 3 * (nn - 1) + 7
    assert extra80 == 19927 and 3 * (nn ** 3 + extra80) == 1654104


def _dense(M):
    return M.toarray()


@pytest.mark.parametrize("kind", ["plane", "patch", "cross"])
def test_structure(kind):
    if kind == "plane":
        s = tiny_system((4, 4, 4))
    elif kind == "patch":
        s = tiny_system((5, 5, 5), [Fracture(1, 2, 1, 4, 1, 4)])
    else:
        s = tiny_system((4, 4, 4), [Fracture(0, 2, 0, 4, 0, 4),
                                    Fracture(1, 2, 0, 4, 0, 4)])
    A = _dense(s.A)
    assert np.array_equal(A, A.T)
    sla.cholesky(A)                                 # A SPD
    assert np.array_equal(_dense(s.C2), _dense(s.C1).T)   # stick: C2 = C1^T
    H = _dense(s.H)
    assert np.array_equal(H, H.T)
    ev = np.linalg.eigvalsh(H)
    assert ev.min() > -1e-12 * ev.max()             # SPSD
    assert abs(ev).min() < 1e-12 * ev.max()         # singular
    # constant traction per component lies in the null space of H
    for f in range(len(s.fractures)):
        faces = np.flatnonzero(s.face_frac == f)
        for c in range(3):
            v = np.zeros(s.n_t)
            v[3 * faces + c] = 1.0
            assert np.abs(H @ v).max() < 1e-12 * np.abs(H).max()
    T = _dense(s.T)
    assert np.array_equal(T, T.T)
    sla.cholesky(T)                                 # T SPD
    # at most 5-point stencil on a single planar fracture
    if kind != "cross":
        assert (np.diff(s.T.indptr) <= 5).all()
    assert s.Q2.nnz == 0
    # traction and pressure are never coupled directly
    J = s.jacobian().toarray()
    nu, nt = s.n_u, s.n_t
    assert not J[nu:nu + nt, nu + nt:].any()
    assert not J[nu + nt:, nu:nu + nt].any()
    # Q1 is minus the normal column of C1
    assert np.array_equal(_dense(s.Q1), -_dense(s.C1)[:, 0::3])


def test_dirichlet_rows():
    s = tiny_system((3, 3, 3))
    d = np.flatnonzero(s.dirichlet)
    A = s.A.tocsr()
    for i in d:
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        assert list(cols) == [i]
    assert s.C1[d].nnz == 0 and s.C2[:, d].nnz == 0
    assert not s.b[d].any()


def test_patch_uniform_strain():
    """u = (0, 0, G z) gives a uniform stress; with t = sigma n on the
    fracture faces (local frame) and p = 0 the first two block rows of J
    reproduce the consistent outer-boundary tractions exactly."""
    for fr, shape in (([Fracture(0, 2, 0, 4, 0, 4)], (4, 4, 4)),
                      ([Fracture(1, 2, 1, 4, 1, 4)], (5, 5, 5)),
                      ([Fracture(0, 2, 0, 4, 0, 4),
                        Fracture(2, 2, 0, 4, 0, 4)], (4, 4, 4))):
        s = tiny_system(shape, fr, uniform_E=True)
        E = s.E[0]
        lam = E * POISSON / ((1 + POISSON) * (1 - 2 * POISSON))
        mu = E / (2 * (1 + POISSON))
        G = 1e-3
        sig = np.array([lam * G, lam * G, (lam + 2 * mu) * G])
        x = np.zeros(s.N)
        x[2:s.n_u:3] = G * s.coords[:, 2]
        tl = np.zeros((s.n_p, 3))
        tl[:, 0] = sig[s.face_axis]           # (N, T1, T2) = (sigma_aa, 0, 0)
        x[s.n_u:s.n_u + s.n_t] = tl.ravel()
        r = s.jacobian() @ x
        # consistent outer tractions on x=0,1 / y=0,1 / z=1
        f = np.zeros(s.n_u)
        conn = s.extras["conn"]
        nx, ny, nz = s.shape
        cells = np.arange(nx * ny * nz)
        ci, cj, ck = cells % nx, (cells // nx) % ny, cells // (nx * ny)
        q = s.h * s.h / 4.0
        for ax, idx, n_ax in ((0, ci, nx), (1, cj, ny), (2, ck, nz)):
            for side in (0, 1):
                if ax == 2 and side == 0:
                    continue                   # fixed bottom
                sel = cells[idx == (n_ax - 1 if side else 0)]
                sign = 1.0 if side else -1.0
                for l in range(8):
                    if ((l >> ax) & 1) != side:
                        continue
                    np.add.at(f, 3 * conn[sel, l] + ax, sign * sig[ax] * q)
        f[s.dirichlet] = 0.0
        scale = np.abs(f).max()
        assert np.abs(r[:s.n_u] - f).max() < 1e-11 * scale
        assert np.abs(r[s.n_u:s.n_u + s.n_t]).max() < 1e-11 * scale
        assert np.abs(r[s.n_u + s.n_t:]).max() == 0.0


def test_seed_determinism():
    a = tiny_system((4, 4, 4), slip_p=0.5, seed=3)
    b = tiny_system((4, 4, 4), slip_p=0.5, seed=3)
    c = tiny_system((4, 4, 4), slip_p=0.5, seed=4)
    for k in ("A", "C1", "Q1", "C2", "H", "T"):
        Ma, Mb = getattr(a, k), getattr(b, k)
        assert np.array_equal(Ma.indptr, Mb.indptr)
        assert np.array_equal(Ma.indices, Mb.indices)
        assert np.array_equal(Ma.data, Mb.data)
    assert np.array_equal(a.b, b.b)
    assert not np.array_equal(a.A.data, c.A.data)


def test_slip_blocks():
    """Slip faces: C2 != C1^T, H non-symmetric, and every 3x3 diagonal
    face block of H (the surrogate H~) invertible."""
    s = tiny_system((4, 4, 4), slip_p=0.5, seed=1)
    assert (s.face_state == 1).any()
    assert abs(s.C2 - s.C1.T).max() > 0
    H = s.H.toarray()
    assert not np.array_equal(H, H.T)
    for K in range(s.n_p):
        blk = H[3 * K:3 * K + 3, 3 * K:3 * K + 3]
        assert abs(np.linalg.det(blk)) > 0


def _open_residual(s, u):
    """Pressure residual of the open-face model at displacement u: storage
    |K| g_K / dt on open faces plus the TPFA fluxes T(Upsilon(g)) p at the
    linearisation pressure, with g_K = g0_K - (Q1^T u)_K / |K| and the cubic
    law Upsilon_K = Upsilon0_K (g_K / g0_K)^3 on open faces."""
    from fracgen.problem import assemble_T, DT
    area = s.h * s.h
    g0 = s.extras["aperture"]
    opn = s.face_state == 2
    g = g0 - (s.Q1.T @ u) / area
    ups = np.where(opn, s.upsilon * (g / g0) ** 3, s.upsilon)
    storage = np.where(opn, area * g / DT, 0.0)
    return storage + assemble_T(s, ups) @ s.extras["p_state"]


@pytest.mark.parametrize("name", ["tiny_open", "c1o"])
def test_open_face_q2_is_the_residual_derivative(name):
    """Q2 (eq. Q2def / Q2vsQ1) against central differences of the pressure
    residual along random displacement directions."""
    if name == "tiny_open":
        s = fracgen.tiny_system((4, 4, 4), slip_p=0.3, open_p=0.4, seed=3)
    else:
        s = fracgen.make_config(name)
    assert (s.face_state == 2).any() and s.Q2.nnz > 0
    rng = np.random.default_rng(0)
    for _ in range(3):
        v = rng.standard_normal(s.n_u)
        v[s.dirichlet] = 0.0
        eps = 1e-7
        fd = (_open_residual(s, eps * v) - _open_residual(s, -eps * v)) / (2 * eps)
        q2v = s.Q2 @ v
        assert np.linalg.norm(fd - q2v) <= 1e-7 * np.linalg.norm(q2v)


def test_open_faces_decouple_the_traction_rows():
    """Open faces: C2 rows vanish, H is -|K|/k I per face with no edge
    stabilization, and stick / slip faces keep their rows."""
    s = fracgen.make_config("c1o")
    opn = np.flatnonzero(s.face_state == 2)
    rows = np.concatenate([3 * opn, 3 * opn + 1, 3 * opn + 2])
    assert np.abs(s.C2[rows]).sum() == 0.0
    H = s.H.tocsr()
    for K in opn:
        blk = H[3 * K:3 * K + 3].toarray()
        diag = blk[:, 3 * K:3 * K + 3]
        assert np.allclose(diag, diag[0, 0] * np.eye(3)) and diag[0, 0] < 0
        off = blk.copy()
        off[:, 3 * K:3 * K + 3] = 0.0
        assert not off.any()
    closed = np.flatnonzero(s.face_state != 2)
    assert np.abs(s.C2[3 * closed]).sum() > 0
