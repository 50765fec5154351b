"""Structured hexahedral meshes with mesh-aligned fractures, and assembly of
the stabilized 3x3 block Jacobian.

Notation follows Sec. 2 of the paper: displacement ``u`` on mesh nodes
(global frame, Q1 finite elements), traction ``t`` (three per fracture face,
face-local frame ``(N, T1, T2)``) and pressure ``p`` (one per face).  The
blocks are those of eq. block_def:

* ``A``  -- elastic stiffness (Q1, 2x2x2 Gauss, per-element Young modulus),
* ``C1`` -- ``([[eta_i]], mu_j)`` over the fracture faces,
* ``Q1`` -- ``-([[eta_i . n]], chi_j)``,
* ``C2`` -- ``C1^T`` on stick faces, the linearised Coulomb rows on slip faces,
* ``H``  -- the jump stabilization ``j_t`` (eq. jump_bilinear_form) plus the
  slip terms,
* ``Q2`` -- ``-Psi(Q1^T)/dt + F_u`` on open faces and their neighbours
  (empty without open faces),
* ``T``  -- the TPFA transmissibility (eq. FV_inner_product) plus
  ``j_p / dt``.

Readings of points the paper leaves open (node splitting, the stabilization
tensor, the slip derivatives, the pressure Dirichlet edges) are fixed here
and listed in the design notes of the repository.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp

# Model constants (Sec. 4 of the paper: dt = 0.5 s, friction angle 30 deg,
# zero cohesion, sigma0 = 10 MPa; Poisson ratio 0.25).
DT = 0.5
TAN_THETA = float(np.tan(np.deg2rad(30.0)))
POISSON = 0.25
SIGMA0 = 10.0
# Scaling of the isotropic stabilization tensor Upsilon^(e) = GAMMA h^3/E I.
GAMMA_STAB = 0.25
APERTURE_REF = 1e-3      # m, opening of open faces when none is given
P_STATE = 0.01           # MPa, amplitude of the linearisation pressure


@dataclass
class Fracture:
    """A rectangle of mesh faces normal to ``axis`` at node plane ``plane``.

    The in-plane axes are ``b = (axis+1) % 3`` and ``c = (axis+2) % 3``;
    the rectangle covers cells ``[b0, b1) x [c0, c1)`` of those axes.
    """
    axis: int
    plane: int
    b0: int
    b1: int
    c0: int
    c1: int

    @property
    def nb(self) -> int:
        return self.b1 - self.b0

    @property
    def nc(self) -> int:
        return self.c1 - self.c0

    @property
    def nfaces(self) -> int:
        return self.nb * self.nc


@dataclass
class BlockSystem:
    """The block Jacobian, one right-hand side and the geometry behind them."""
    name: str
    shape: Tuple[int, int, int]
    h: float
    n_u: int
    n_t: int
    n_p: int
    A: sp.csr_matrix
    C1: sp.csr_matrix
    Q1: sp.csr_matrix
    C2: sp.csr_matrix
    H: sp.csr_matrix
    Q2: sp.csr_matrix
    T: sp.csr_matrix
    b: np.ndarray
    coords: np.ndarray            # (n_u/3, 3) node coordinates (copies repeat)
    dirichlet: np.ndarray         # (n_u,) bool
    n_nodes_orig: int
    fractures: List[Fracture]
    face_frac: np.ndarray         # (n_p,) fracture id of each face
    face_axis: np.ndarray         # (n_p,) normal axis
    face_cells: np.ndarray        # (n_p, 2) minus / plus cell
    face_state: np.ndarray        # (n_p,) 0 stick, 1 slip
    slip_dir: np.ndarray          # (n_p, 2) unit tangent in (T1, T2)
    E: np.ndarray                 # (n_cells,) Young modulus
    upsilon: np.ndarray           # (n_p,) one-sided transmissibility
    flow_pairs: np.ndarray        # (m, 2) TPFA face pairs (K < L)
    flow_ndir: np.ndarray         # (n_p,) number of Dirichlet edges
    stab_pairs: np.ndarray        # (s, 2) coplanar same-fracture face pairs
    stab_weight: np.ndarray       # (s,) gamma h^3 / E_bar per pair
    T_stab: sp.csr_matrix         # j_p / dt part of T (independent of Upsilon)
    seed: int = 0
    extras: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n_u + self.n_t + self.n_p

    def jacobian(self) -> sp.csr_matrix:
        """The assembled ``J = [A C1 Q1; C2 -H 0; Q2 0 T]`` (eq. JacSys)."""
        J = sp.bmat([[self.A, self.C1, self.Q1],
                     [self.C2, -self.H, None],
                     [self.Q2, None, self.T]], format="csr")
        J.sort_indices()
        return J

    def blocks(self):
        return dict(A=self.A, C1=self.C1, Q1=self.Q1, C2=self.C2, H=self.H,
                    Q2=self.Q2, T=self.T)


# ----------------------------------------------------------------------------
# Element matrices
# ----------------------------------------------------------------------------

def reference_stiffness(nu: float = POISSON) -> np.ndarray:
    """24x24 stiffness of the unit-cube Q1 element for E = 1.

    Local node ``l = cx + 2 cy + 4 cz``; dof ``3 l + component``.  For a cube
    of side ``h`` and modulus ``E`` the element matrix is ``E h`` times this.
    """
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1.0 / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    for i in range(3):
        D[i, i] = lam + 2 * mu
        D[3 + i, 3 + i] = mu
    gp = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]
    K = np.zeros((24, 24))
    for x in gp:
        for y in gp:
            for z in gp:
                B = np.zeros((6, 24))
                for l in range(8):
                    cx, cy, cz = l & 1, (l >> 1) & 1, (l >> 2) & 1
                    fx, dfx = (x, 1.0) if cx else (1 - x, -1.0)
                    fy, dfy = (y, 1.0) if cy else (1 - y, -1.0)
                    fz, dfz = (z, 1.0) if cz else (1 - z, -1.0)
                    dx, dy, dz = dfx * fy * fz, fx * dfy * fz, fx * fy * dfz
                    B[0, 3 * l] = dx
                    B[1, 3 * l + 1] = dy
                    B[2, 3 * l + 2] = dz
                    B[3, 3 * l + 1] = dz
                    B[3, 3 * l + 2] = dy
                    B[4, 3 * l] = dz
                    B[4, 3 * l + 2] = dx
                    B[5, 3 * l] = dy
                    B[5, 3 * l + 1] = dx
                K += 0.125 * B.T @ D @ B
    K = 0.5 * (K + K.T)
    K[np.abs(K) < 1e-14 * np.abs(K).max()] = 0.0
    return K


# ----------------------------------------------------------------------------
# Helpers
# ----------------------------------------------------------------------------

def _csr(rows, cols, vals, shape) -> sp.csr_matrix:
    M = sp.coo_matrix((vals, (rows, cols)), shape=shape).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    return M


def _canon(M: sp.csr_matrix) -> sp.csr_matrix:
    M = sp.csr_matrix(M)
    M.sum_duplicates()
    M.sort_indices()
    return M


class _Grid:
    def __init__(self, shape, h):
        self.n = np.asarray(shape, dtype=np.int64)
        self.h = float(h)
        self.nn = self.n + 1

    def node(self, idx):
        i, j, k = idx
        return i + self.nn[0] * (j + self.nn[1] * k)

    def cell(self, idx):
        i, j, k = idx
        return i + self.n[0] * (j + self.n[1] * k)

    @property
    def n_nodes(self):
        return int(np.prod(self.nn))

    @property
    def n_cells(self):
        return int(np.prod(self.n))


def _face_index_arrays(fr: Fracture):
    """Per-face (ib, ic) of a fracture in the face order (b fastest)."""
    ic, ib = np.meshgrid(np.arange(fr.c0, fr.c1), np.arange(fr.b0, fr.b1),
                         indexing="ij")
    return ib.ravel(), ic.ravel()


def _idx3(axis, av, bv, cv):
    """Assemble (i, j, k) from values along (axis, axis+1, axis+2)."""
    out = [None, None, None]
    out[axis] = av
    out[(axis + 1) % 3] = bv
    out[(axis + 2) % 3] = cv
    return out


# ----------------------------------------------------------------------------
# Main builder
# ----------------------------------------------------------------------------

def build_system(shape: Sequence[int], h: float, fractures: List[Fracture],
                 E: np.ndarray, upsilon: np.ndarray,
                 face_state: Optional[np.ndarray] = None,
                 slip_angle: Optional[np.ndarray] = None,
                 q: Optional[np.ndarray] = None, name: str = "custom",
                 seed: int = 0, top_load: bool = True,
                 aperture: Optional[np.ndarray] = None) -> BlockSystem:
    """Assemble the block system on an ``nx x ny x nz`` grid of cubes.

    ``E`` holds one Young modulus per cell (cell id ``i + nx (j + ny k)``),
    ``upsilon`` one transmissibility per fracture face, ``face_state`` 0
    (stick), 1 (slip) or 2 (open) per face, ``slip_angle`` the angle of the
    slip direction in the (T1, T2) plane, ``q`` the pressure source (``b_p =
    q / |q|``) and ``aperture`` the current normal opening of every face
    (used on open faces only; default ``APERTURE_REF``).
    """
    g = _Grid(shape, h)
    nx, ny, nz = (int(v) for v in g.n)
    n_cells = g.n_cells
    n_nodes0 = g.n_nodes

    # ---------------- fracture faces --------------------------------------
    fmark = {}
    for a in range(3):
        sh = [int(v) for v in g.n]
        sh[a] += 1
        fmark[a] = np.zeros(sh, dtype=bool)
    face_frac, face_axis, face_ib, face_ic, face_plane = [], [], [], [], []
    for f, fr in enumerate(fractures):
        a = fr.axis
        if not (1 <= fr.plane <= int(g.n[a]) - 1):
            raise ValueError("fracture plane must be interior")
        nbv, ncv = int(g.n[(a + 1) % 3]), int(g.n[(a + 2) % 3])
        if not (0 <= fr.b0 < fr.b1 <= nbv and 0 <= fr.c0 < fr.c1 <= ncv):
            raise ValueError("fracture extent out of range")
        if fr.nb < 2 or fr.nc < 2:
            raise ValueError("fractures need at least 2x2 faces")
        ib, ic = _face_index_arrays(fr)
        idx = _idx3(a, np.full_like(ib, fr.plane), ib, ic)
        if fmark[a][tuple(idx)].any():
            raise ValueError("overlapping fractures")
        fmark[a][tuple(idx)] = True
        face_frac.append(np.full(ib.size, f))
        face_axis.append(np.full(ib.size, a))
        face_ib.append(ib)
        face_ic.append(ic)
        face_plane.append(np.full(ib.size, fr.plane))
    face_frac = np.concatenate(face_frac).astype(np.int64)
    face_axis = np.concatenate(face_axis).astype(np.int64)
    face_ib = np.concatenate(face_ib).astype(np.int64)
    face_ic = np.concatenate(face_ic).astype(np.int64)
    face_plane = np.concatenate(face_plane).astype(np.int64)
    n_p = face_frac.size
    n_t = 3 * n_p

    # minus / plus cells and the four corner nodes (db, dc) of every face
    minus_cell = np.empty(n_p, np.int64)
    plus_cell = np.empty(n_p, np.int64)
    corner_nodes = np.empty((n_p, 4), np.int64)
    corner_d = [(0, 0), (1, 0), (0, 1), (1, 1)]
    for a in range(3):
        m = face_axis == a
        if not m.any():
            continue
        pl, ib, ic = face_plane[m], face_ib[m], face_ic[m]
        minus_cell[m] = g.cell(_idx3(a, pl - 1, ib, ic))
        plus_cell[m] = g.cell(_idx3(a, pl, ib, ic))
        for j, (db, dc) in enumerate(corner_d):
            corner_nodes[m, j] = g.node(_idx3(a, pl, ib + db, ic + dc))

    # ---------------- node splitting ---------------------------------------
    # Each node gets one copy per class of its incident cells connected
    # through non-fracture faces.  The class holding the lowest local cell
    # keeps the original id; the other copies are appended, ordered by
    # (original node, class).
    cand = np.unique(corner_nodes.ravel())
    ci = cand % g.nn[0]
    cj = (cand // g.nn[0]) % g.nn[1]
    ck = cand // (g.nn[0] * g.nn[1])
    cidx = np.stack([ci, cj, ck], axis=1)
    nc_ = cand.size
    exists = np.zeros((nc_, 8), bool)
    for o in range(8):
        off = np.array([(o >> d) & 1 for d in range(3)]) - 1
        c3 = cidx + off
        exists[:, o] = np.all((c3 >= 0) & (c3 < g.n), axis=1)
    edges = []
    for o in range(8):
        for d in range(3):
            if (o >> d) & 1 == 0:
                edges.append((o, o | (1 << d), d))
    conn_e = np.zeros((nc_, len(edges)), bool)
    for e_, (o1, o2, d) in enumerate(edges):
        both = exists[:, o1] & exists[:, o2]
        # the face between the two cells: node plane along d, cell index
        # (node - 1 + o) along the other axes (o1 and o2 agree there)
        fidx = []
        for ax in range(3):
            if ax == d:
                fidx.append(cidx[:, ax])
            else:
                fidx.append(cidx[:, ax] - 1 + ((o1 >> ax) & 1))
        fidx = [np.where(both, v, 0) for v in fidx]
        isfrac = fmark[d][tuple(fidx)]
        conn_e[:, e_] = both & ~isfrac
    lab = np.where(exists, np.arange(8)[None, :], 99)
    for _ in range(8):
        old = lab.copy()
        for e_, (o1, o2, d) in enumerate(edges):
            c = conn_e[:, e_]
            mn = np.minimum(lab[:, o1], lab[:, o2])
            lab[c, o1] = mn[c]
            lab[c, o2] = mn[c]
        if np.array_equal(old, lab):
            break
    is_rep = exists & (lab == np.arange(8)[None, :])
    nrep = is_rep.sum(axis=1)
    first_rep = np.argmax(is_rep, axis=1)
    extra_mask = is_rep.copy()
    extra_mask[np.arange(nc_), first_rep] = False
    n_extra = int(extra_mask.sum())
    copy_id = np.full((nc_, 8), -1, np.int64)
    copy_id[np.arange(nc_), first_rep] = cand
    copy_id[extra_mask] = n_nodes0 + np.arange(n_extra)   # row-major order
    node_of_cell = np.where(exists, np.take_along_axis(
        copy_id, np.where(exists, lab, 0), axis=1), -1)
    n_nodes = n_nodes0 + n_extra
    orig_of_node = np.concatenate([
        np.arange(n_nodes0),
        np.repeat(cand, 8)[extra_mask.ravel()]])
    assert orig_of_node.size == n_nodes
    del nrep

    # element connectivity with split copies
    cells = np.arange(n_cells)
    cxi = cells % nx
    cyj = (cells // nx) % ny
    czk = cells // (nx * ny)
    conn = np.empty((n_cells, 8), np.int64)
    is_cand = np.zeros(n_nodes0, bool)
    is_cand[cand] = True
    cand_pos = np.full(n_nodes0, -1, np.int64)
    cand_pos[cand] = np.arange(nc_)
    for l in range(8):
        cx, cy, cz = l & 1, (l >> 1) & 1, (l >> 2) & 1
        nd = g.node((cxi + cx, cyj + cy, czk + cz))
        sel = is_cand[nd]
        nd = nd.copy()
        nd[sel] = node_of_cell[cand_pos[nd[sel]], 7 - l]
        conn[:, l] = nd

    oi = orig_of_node % g.nn[0]
    oj = (orig_of_node // g.nn[0]) % g.nn[1]
    ok = orig_of_node // (g.nn[0] * g.nn[1])
    coords = np.stack([oi, oj, ok], axis=1).astype(np.float64) * g.h
    n_u = 3 * n_nodes
    dir_node = ok == 0
    dirichlet = np.repeat(dir_node, 3)

    # ---------------- A: elastic stiffness ---------------------------------
    E = np.asarray(E, dtype=np.float64)
    assert E.shape == (n_cells,)
    Kref = reference_stiffness()
    A = _assemble_stiffness(conn, E * g.h, Kref, n_nodes)
    # exact symmetry: the element sums reach (i, j) and (j, i) in different
    # orders; (a + b) / 2 is order independent
    A = ((A + A.T) * 0.5).tocsr()
    A = _dirichlet_sym(A, dirichlet)

    # ---------------- C1, Q1 -------------------------------------------------
    rows, cols, vals = [], [], []
    areaq = g.h * g.h / 4.0
    for j, (db, dc) in enumerate(corner_d):
        for side, cellarr, sgn in ((0, minus_cell, -1.0), (1, plus_cell, 1.0)):
            # local corner of the cell: along the normal axis the minus cell
            # sees the face at its upper side, the plus cell at its lower side
            lcorner = np.zeros(n_p, np.int64)
            for a in range(3):
                m = face_axis == a
                la = (1 << a) if side == 0 else 0
                lcorner[m] = la + (db << ((a + 1) % 3)) + (dc << ((a + 2) % 3))
            node = conn[cellarr, lcorner]
            for ld in range(3):
                comp = (face_axis + ld) % 3
                rows.append(3 * node + comp)
                cols.append(3 * np.arange(n_p) + ld)
                vals.append(np.full(n_p, sgn * areaq))
    C1 = _csr(np.concatenate(rows), np.concatenate(cols),
              np.concatenate(vals), (n_u, n_t))
    C1.eliminate_zeros()           # tip nodes: equal +/- copies cancel exactly
    C1 = _zero_rows(C1, dirichlet)
    Q1 = _canon(-C1[:, 0::3])

    # ---------------- stabilization edges ----------------------------------
    stab_pairs, stab_w = [], []
    for f, fr in enumerate(fractures):
        base = np.flatnonzero(face_frac == f)[0]
        nb, ncc = fr.nb, fr.nc
        loc = np.arange(nb * ncc).reshape(ncc, nb)
        pk = np.concatenate([loc[:, :-1].ravel(), loc[:-1, :].ravel()]) + base
        pl_ = np.concatenate([loc[:, 1:].ravel(), loc[1:, :].ravel()]) + base
        stab_pairs.append(np.stack([pk, pl_], axis=1))
    stab_pairs = np.concatenate(stab_pairs).astype(np.int64)
    K_, L_ = stab_pairs[:, 0], stab_pairs[:, 1]
    inv_sum = (1.0 / E[minus_cell[K_]] + 1.0 / E[plus_cell[K_]]
               + 1.0 / E[minus_cell[L_]] + 1.0 / E[plus_cell[L_]])
    Ebar = 4.0 / inv_sum
    stab_w = GAMMA_STAB * g.h ** 3 / Ebar
    s_face = np.bincount(K_, stab_w, n_p) + np.bincount(L_, stab_w, n_p)

    # ---------------- states, H and C2 --------------------------------------
    if face_state is None:
        face_state = np.zeros(n_p, np.int64)
    face_state = np.asarray(face_state, np.int64).copy()
    if (face_state == 2).any():
        # a stick / slip face none of whose coplanar neighbours is closed has
        # no edge for j_t: its block of Bdiag(H, 3) would vanish; such an
        # island inside an open region is taken as open
        closed = face_state != 2
        n_closed = (np.bincount(K_, closed[L_], n_p)
                    + np.bincount(L_, closed[K_], n_p))
        face_state[closed & (n_closed == 0)] = 2
    if slip_angle is None:
        slip_angle = np.zeros(n_p)
    slip_dir = np.stack([np.cos(slip_angle), np.sin(slip_angle)], axis=1)

    is_open = face_state == 2
    # j_t acts on edges between stick / slip faces only (eq. Hdef)
    closed_edge = ~is_open[K_] & ~is_open[L_]
    Kc, Lc, wc = K_[closed_edge], L_[closed_edge], stab_w[closed_edge]
    hr, hc, hv = [], [], []
    for ld in range(3):
        hr += [3 * Kc + ld, 3 * Lc + ld, 3 * Kc + ld, 3 * Lc + ld]
        hc += [3 * Kc + ld, 3 * Lc + ld, 3 * Lc + ld, 3 * Kc + ld]
        hv += [wc, wc, -wc, -wc]
    opn = np.flatnonzero(is_open)
    if opn.size:
        # -(1/k)(mu_i, mu_j) on open faces: -|K|/k_K = -2 s_K, all components
        for ld in range(3):
            hr.append(3 * opn + ld)
            hc.append(3 * opn + ld)
            hv.append(-2.0 * s_face[opn])
    slip = np.flatnonzero(face_state == 1)
    if slip.size:
        # (1/k) terms with k_K = |K| / (2 s_K): -2 s_K on TT and
        # -2 s_K tan(theta) d on TN
        for i in range(2):
            hr += [3 * slip + 1 + i, 3 * slip + 1 + i]
            hc += [3 * slip + 1 + i, 3 * slip]
            hv += [-2.0 * s_face[slip],
                   -2.0 * s_face[slip] * TAN_THETA * slip_dir[slip, i]]
    H = _csr(np.concatenate(hr), np.concatenate(hc), np.concatenate(hv),
             (n_t, n_t))

    # slip tangential rows: -(I - d d^T) applied to the C1^T (T1, T2) rows
    C1T = sp.csr_matrix(C1.T)
    if slip.size:
        d = slip_dir[slip]
        Pm = np.eye(2)[None] - d[:, :, None] * d[:, None, :]
        keep = np.ones(n_t, bool)
        keep[3 * slip + 1] = False
        keep[3 * slip + 2] = False
        mr = [np.flatnonzero(keep)]
        mc = [np.flatnonzero(keep)]
        mv = [np.ones(int(keep.sum()))]
        for i in range(2):
            for j in range(2):
                mr.append(3 * slip + 1 + i)
                mc.append(3 * slip + 1 + j)
                mv.append(-Pm[:, i, j])
        Mrow = _csr(np.concatenate(mr), np.concatenate(mc),
                    np.concatenate(mv), (n_t, n_t))
        C2 = Mrow @ C1T
    else:
        C2 = C1T
    if opn.size:
        # no traction-jump coupling on open faces (eq. C2def)
        keep_rows = np.ones(n_t)
        keep_rows[np.concatenate([3 * opn, 3 * opn + 1, 3 * opn + 2])] = 0.0
        C2 = sp.diags(keep_rows) @ C2
    C2 = _canon(C2)

    # ---------------- T: TPFA + j_p/dt + Dirichlet -------------------------
    ekeys, efaces = [], []
    for a in range(3):
        m = np.flatnonzero(face_axis == a)
        if m.size == 0:
            continue
        pl, ib, ic = face_plane[m], face_ib[m], face_ic[m]
        b_ax, c_ax = (a + 1) % 3, (a + 2) % 3
        # edges along b at c = ic and c = ic + 1; along c at b = ib, ib + 1
        for (dbb, dcc, dirax) in ((0, 0, b_ax), (0, 1, b_ax),
                                  (0, 0, c_ax), (1, 0, c_ax)):
            nd = g.node(_idx3(a, pl, ib + dbb, ic + dcc))
            ekeys.append(3 * nd + dirax)
            efaces.append(m)
    ekeys = np.concatenate(ekeys)
    efaces = np.concatenate(efaces)
    order = np.lexsort((efaces, ekeys))
    ekeys, efaces = ekeys[order], efaces[order]
    starts = np.flatnonzero(np.r_[True, ekeys[1:] != ekeys[:-1]])
    sizes = np.diff(np.r_[starts, ekeys.size])
    fp = []
    for gsz in np.unique(sizes):
        if gsz < 2:
            continue
        st = starts[sizes == gsz]
        for x in range(gsz):
            for y in range(x + 1, gsz):
                fp.append(np.stack([efaces[st + x], efaces[st + y]], axis=1))
    flow_pairs = np.concatenate(fp) if fp else np.zeros((0, 2), np.int64)
    flow_pairs = np.sort(flow_pairs, axis=1)
    flow_pairs = np.unique(flow_pairs, axis=0)

    flow_ndir = np.zeros(n_p, np.int64)
    for f, fr in enumerate(fractures):
        base = np.flatnonzero(face_frac == f)[0]
        nb, ncc = fr.nb, fr.nc
        for (x, y) in ((0, 0), (nb - 1, 0), (0, ncc - 1), (nb - 1, ncc - 1)):
            flow_ndir[base + y * nb + x] += 2

    T_stab = _laplacian(stab_pairs, stab_w / DT, n_p)
    upsilon = np.asarray(upsilon, np.float64)
    assert upsilon.shape == (n_p,)

    # ---------------- open faces: Q2 (eq. Q2def, eq. Q2vsQ1) ----------------
    if aperture is None:
        aperture = np.full(n_p, APERTURE_REF)
    aperture = np.asarray(aperture, np.float64)
    centre = np.zeros((n_p, 3))
    for a in range(3):
        m = face_axis == a
        centre[m, a] = face_plane[m] * g.h
        centre[m, (a + 1) % 3] = (face_ib[m] + 0.5) * g.h
        centre[m, (a + 2) % 3] = (face_ic[m] + 0.5) * g.h
    p_state = pressure_state(centre)
    Q2 = open_face_q2(Q1, face_state, upsilon, aperture, p_state, flow_pairs,
                      flow_ndir, g.h * g.h)

    # ---------------- right-hand side ---------------------------------------
    b = np.zeros(n_u + n_t + n_p)
    if top_load:
        top = np.flatnonzero(czk == nz - 1)
        for l in (4, 5, 6, 7):
            np.add.at(b, 3 * conn[top, l] + 2, -SIGMA0 * g.h * g.h / 4.0)
    b[:n_u][dirichlet] = 0.0
    if q is None:
        q = np.zeros(n_p)
    qn = np.linalg.norm(q)
    if qn > 0:
        b[n_u + n_t:] = q / qn

    sysm = BlockSystem(
        name=name, shape=tuple(int(v) for v in g.n), h=g.h, n_u=n_u, n_t=n_t,
        n_p=n_p, A=_canon(A), C1=_canon(C1), Q1=Q1, C2=C2, H=_canon(H),
        Q2=Q2, T=None, b=b, coords=coords,
        dirichlet=dirichlet, n_nodes_orig=n_nodes0, fractures=list(fractures),
        face_frac=face_frac, face_axis=face_axis,
        face_cells=np.stack([minus_cell, plus_cell], axis=1),
        face_state=face_state, slip_dir=slip_dir, E=E, upsilon=upsilon,
        flow_pairs=flow_pairs.astype(np.int64), flow_ndir=flow_ndir,
        stab_pairs=stab_pairs, stab_weight=stab_w, T_stab=T_stab, seed=seed)
    sysm.T = assemble_T(sysm, upsilon)
    sysm.extras["conn"] = conn
    sysm.extras["aperture"] = aperture
    sysm.extras["p_state"] = p_state
    sysm.extras["face_centre"] = centre
    sysm.extras["orig_of_node"] = orig_of_node
    return sysm


def _laplacian(pairs, w, n):
    K, L = pairs[:, 0], pairs[:, 1]
    r = np.concatenate([K, L, K, L])
    c = np.concatenate([K, L, L, K])
    v = np.concatenate([w, w, -w, -w])
    return _canon(_csr(r, c, v, (n, n)))


def pressure_state(centre: np.ndarray) -> np.ndarray:
    """The current fracture pressure the Newton step linearises about (a
    smooth synthetic field, amplitude ``P_STATE``), per face centre."""
    x, y, z = centre[:, 0], centre[:, 1], centre[:, 2]
    return P_STATE * (np.cos(2 * np.pi * x) * np.cos(2 * np.pi * y)
                      * np.cos(2 * np.pi * z))


def open_face_q2(Q1, face_state, upsilon, aperture, p_state, flow_pairs,
                 flow_ndir, area) -> sp.csr_matrix:
    """``Q2 = -Psi(Q1^T)/dt + F_u`` (eq. Q2vsQ1).

    The storage term of an open face K, ``|K| g_K / dt`` with the
    face-averaged opening ``g_K = -(Q1^T u)_K / |K|``, gives ``-Q1^T/dt`` on
    the open rows.  ``F_u`` is the derivative of the TPFA fluxes
    (eq. FV_inner_product) at the pressure state ``p_state`` through the
    cubic law ``Upsilon_K ~ g_K^3`` on open faces: ``dUpsilon_K / dg_K =
    3 Upsilon_K / g_K``, chained through the harmonic average.  Rows of
    faces without an open neighbour and without opening are empty.
    """
    n_p = face_state.size
    n_u = Q1.shape[0]
    is_open = face_state == 2
    if not is_open.any():
        return _canon(sp.csr_matrix((n_p, n_u)))
    Q1T = sp.csr_matrix(Q1.T)
    G = -Q1T / area                               # row K: d g_K / d u
    dU = np.where(is_open, 3.0 * upsilon / aperture, 0.0)
    K, L = flow_pairs[:, 0], flow_pairs[:, 1]
    uK, uL = upsilon[K], upsilon[L]
    den = (uK + uL) ** 2
    cK = 2.0 * uL * uL / den * dU[K]             # d U_KL / d g_K
    cL = 2.0 * uK * uK / den * dU[L]             # d U_KL / d g_L
    dp = p_state[L] - p_state[K]
    # flux row K: -U_KL (p_L - p_K); row L: +U_KL (p_L - p_K); Dirichlet
    # edges: n_dir U_K p_K
    rows = np.concatenate([K, K, L, L, np.arange(n_p)])
    cols = np.concatenate([K, L, K, L, np.arange(n_p)])
    vals = np.concatenate([-dp * cK, -dp * cL, dp * cK, dp * cL,
                           flow_ndir * p_state * dU])
    W = sp.csr_matrix((vals, (rows, cols)), shape=(n_p, n_p))
    W.eliminate_zeros()
    storage = sp.diags(np.where(is_open, -1.0 / DT, 0.0)) @ Q1T
    return _canon(sp.csr_matrix(storage + W @ G))


def transmissibility_pairs(upsilon: np.ndarray, pairs: np.ndarray):
    """Harmonic average 2 U_K U_L / (U_K + U_L) of the one-sided values."""
    uK, uL = upsilon[pairs[:, 0]], upsilon[pairs[:, 1]]
    return 2.0 * uK * uL / (uK + uL)


def assemble_T(sysm: BlockSystem, upsilon: np.ndarray) -> sp.csr_matrix:
    """``T(Upsilon)``: TPFA (eq. FV_inner_product) + j_p/dt + Dirichlet."""
    upsilon = np.asarray(upsilon, np.float64)
    n = sysm.n_p
    w = transmissibility_pairs(upsilon, sysm.flow_pairs)
    Tf = _laplacian(sysm.flow_pairs, w, n) if len(w) else sp.csr_matrix((n, n))
    Td = sp.diags(sysm.flow_ndir * upsilon, format="csr")
    T = (Tf + Td + sysm.T_stab).tocsr()
    return _canon(T)


def flow_loss(p: np.ndarray, p_obs: np.ndarray) -> float:
    """Misfit 0.5 |p - p_obs|^2 over the fracture pressures."""
    r = p - p_obs
    return 0.5 * float(r @ r)


def _assemble_stiffness(conn, scale, Kref, n_nodes):
    """Node-block assembly of sum_e scale_e * Kref into a scalar CSR."""
    n_cells = conn.shape[0]
    rows = np.empty((8, 8, n_cells), np.int64)
    cols = np.empty((8, 8, n_cells), np.int64)
    for l in range(8):
        for m in range(8):
            rows[l, m] = conn[:, l]
            cols[l, m] = conn[:, m]
    keys = (rows * n_nodes + cols).ravel()
    del rows, cols
    order = np.argsort(keys, kind="stable")
    ks = keys[order]
    del keys
    uniq_start = np.flatnonzero(np.r_[True, ks[1:] != ks[:-1]])
    ukeys = ks[uniq_start]
    del ks
    # blocks in (l, m, cell) order -> value of entry (r, s) of block
    nb = ukeys.size
    blocks = np.empty((nb, 3, 3))
    lm_of = order // n_cells
    cell_of = order % n_cells
    del order
    l_of = lm_of // 8
    m_of = lm_of % 8
    for r in range(3):
        for s in range(3):
            v = scale[cell_of] * Kref[3 * l_of + r, 3 * m_of + s]
            blocks[:, r, s] = np.add.reduceat(v, uniq_start)
    del lm_of, cell_of, l_of, m_of
    brow = ukeys // n_nodes
    bcol = ukeys % n_nodes
    # scalar CSR: row 3i+r has entries (3j+s) for each block column j
    nblk_row = np.bincount(brow, minlength=n_nodes)
    row_len = np.repeat(3 * nblk_row, 3)
    indptr = np.zeros(3 * n_nodes + 1, np.int64)
    np.cumsum(row_len, out=indptr[1:])
    bstart = np.zeros(n_nodes + 1, np.int64)
    np.cumsum(nblk_row, out=bstart[1:])
    nnz = int(indptr[-1])
    indices = np.empty(nnz, np.int64)
    data = np.empty(nnz)
    # position of block b (row i, k-th in row) entry (r, s):
    #   indptr[3i + r] + 3 k + s
    kpos = np.arange(nb) - bstart[brow]
    for r in range(3):
        base = indptr[3 * brow + r] + 3 * kpos
        for s in range(3):
            indices[base + s] = 3 * bcol + s
            data[base + s] = blocks[:, r, s]
    A = sp.csr_matrix((data, indices, indptr), shape=(3 * n_nodes,) * 2)
    return A


def _dirichlet_sym(A: sp.csr_matrix, dmask: np.ndarray) -> sp.csr_matrix:
    """Keep the diagonal of Dirichlet rows, drop their row/column couplings."""
    A = sp.csr_matrix(A)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    keep = (rows == A.indices) | (~dmask[rows] & ~dmask[A.indices])
    return _filter(A, rows, keep)


def _zero_rows(M: sp.csr_matrix, dmask: np.ndarray) -> sp.csr_matrix:
    M = sp.csr_matrix(M)
    rows = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))
    return _filter(M, rows, ~dmask[rows])


def _filter(M, rows, keep):
    indptr = np.zeros(M.shape[0] + 1, np.int64)
    np.cumsum(np.bincount(rows[keep], minlength=M.shape[0]), out=indptr[1:])
    out = sp.csr_matrix((M.data[keep], M.indices[keep], indptr), shape=M.shape)
    out.sort_indices()
    return out
