"""The five seeded workloads and small test systems.

Every random draw comes from ``numpy.random.PCG64`` streams spawned from one
``SeedSequence(seed)`` in a fixed order: Young modulus, transmissibility,
contact states, slip directions, fracture geometry, right-hand side,
observations.

Workloads (sizes are cells per axis on the unit cube unless noted):

* ``c1``  10^3, one full fracture plane x = 0.5 (100 faces), all stick.
* ``c2``  80^3, full planes x, y, z = 0.5 (19,200 faces), Bernoulli(0.3) slip.
* ``c3``  128 x 128 x 64 on [0,1]^2 x [0,0.5], 12 random rectangles,
  layered modulus (8 layers, contrast 1e3, lognormal noise).
* ``c4``  64^3, 6 random rectangles, 32 right-hand sides.
* ``c5``  48^3, 4 full x-normal planes (9,216 faces), pressure observations.
"""
from __future__ import annotations

from typing import List, Optional, Tuple

import numpy as np
import scipy.sparse.linalg as spla

from .problem import (APERTURE_REF, BlockSystem, Fracture, assemble_T,
                      build_system)

CONFIGS = ("c1", "c2", "c3", "c4", "c5")
# with open faces (eq. Q2vsQ1): the c1 and c2 meshes with part of the faces
# open; not among the five workloads above
OPEN_CONFIGS = ("c1o", "c2o")
TRANS_MEDIAN_SI = 1e-10     # m^3 / (Pa s)
PA_PER_MPA = 1e6


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    names = ("E", "upsilon", "state", "slipdir", "frac", "rhs", "obs", "open")
    return {n: np.random.Generator(np.random.PCG64(s))
            for n, s in zip(names, ss.spawn(len(names)))}


def _lognormal_E(rng, n_cells, median=1e4, sigma=0.5):
    return median * np.exp(sigma * rng.standard_normal(n_cells))


def _layered_E(rng, shape, nlayers=8, contrast=1e3, sigma=0.5):
    """8 z-layers with E_L = 1e4 * contrast^(pi_L/7 - 1/2) and noise."""
    nx, ny, nz = shape
    perm = rng.permutation(nlayers)
    layer_of_k = (np.arange(nz) * nlayers) // nz
    base = 1e4 * contrast ** (perm / (nlayers - 1) - 0.5)
    Ek = base[layer_of_k]
    E = np.broadcast_to(Ek[:, None, None], (nz, ny, nx)).ravel().copy()
    return E * np.exp(sigma * rng.standard_normal(E.size))


def _random_rectangles(rng, shape, count, lo, hi, max_tries=100000):
    """Mesh-aligned rectangles whose node sets are pairwise disjoint."""
    n = np.asarray(shape)
    out: List[Fracture] = []
    boxes = []
    tries = 0
    while len(out) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place fractures")
        a = int(rng.integers(3))
        b, c = (a + 1) % 3, (a + 2) % 3
        sb = int(rng.integers(lo, min(hi, n[b] - 2) + 1))
        sc = int(rng.integers(lo, min(hi, n[c] - 2) + 1))
        b0 = int(rng.integers(1, n[b] - sb))
        c0 = int(rng.integers(1, n[c] - sc))
        pl = int(rng.integers(1, n[a]))
        box = [None, None, None]
        box[a] = (pl, pl)
        box[b] = (b0, b0 + sb)
        box[c] = (c0, c0 + sc)
        clash = any(all(bx[d][0] <= box[d][1] and box[d][0] <= bx[d][1]
                        for d in range(3)) for bx in boxes)
        if clash:
            continue
        boxes.append(box)
        out.append(Fracture(a, pl, b0, b0 + sb, c0, c0 + sc))
    return out


def make_config(name: str, seed: int = 0) -> BlockSystem:
    """Build workload ``name`` (``c1`` ... ``c5``)."""
    rs = _streams(seed)
    if name == "c1":
        shape, h = (10, 10, 10), 0.1
        fr = [Fracture(0, 5, 0, 10, 0, 10)]
        E = _lognormal_E(rs["E"], 1000)
        slip_p = 0.0
    elif name == "c2":
        shape, h = (80, 80, 80), 1.0 / 80
        fr = [Fracture(0, 40, 0, 80, 0, 80), Fracture(1, 40, 0, 80, 0, 80),
              Fracture(2, 40, 0, 80, 0, 80)]
        E = _lognormal_E(rs["E"], 80 ** 3)
        slip_p = 0.3
    elif name == "c3":
        shape, h = (128, 128, 64), 1.0 / 128
        fr = _random_rectangles(rs["frac"], shape, 12, 40, 80)
        E = _layered_E(rs["E"], shape)
        slip_p = 0.0
    elif name == "c4":
        shape, h = (64, 64, 64), 1.0 / 64
        fr = _random_rectangles(rs["frac"], shape, 6, 16, 40)
        E = _lognormal_E(rs["E"], 64 ** 3)
        slip_p = 0.0
    elif name == "c5":
        shape, h = (48, 48, 48), 1.0 / 48
        fr = [Fracture(0, i, 0, 48, 0, 48) for i in (10, 19, 29, 38)]
        E = _lognormal_E(rs["E"], 48 ** 3)
        slip_p = 0.0
    elif name == "c1o":
        shape, h = (10, 10, 10), 0.1
        fr = [Fracture(0, 5, 0, 10, 0, 10)]
        E = _lognormal_E(rs["E"], 1000)
        return _finish(name, shape, h, fr, E, 0.2, rs, seed, open_p=0.3)
    elif name == "c2o":
        shape, h = (80, 80, 80), 1.0 / 80
        fr = [Fracture(0, 40, 0, 80, 0, 80), Fracture(1, 40, 0, 80, 0, 80),
              Fracture(2, 40, 0, 80, 0, 80)]
        E = _lognormal_E(rs["E"], 80 ** 3)
        return _finish(name, shape, h, fr, E, 0.3, rs, seed, open_p=0.1)
    else:
        raise KeyError(name)
    return _finish(name, shape, h, fr, E, slip_p, rs, seed)


def _finish(name, shape, h, fr, E, slip_p, rs, seed, top_load=True,
            open_p=0.0):
    n_p = sum(f.nfaces for f in fr)
    # median 1e-10 m^3/(Pa s) in SI, expressed in the MPa unit system of the
    # mechanics (E in MPa): 1e-10 m^3/(Pa s) = 1e-4 m^3/(MPa s)
    ups = TRANS_MEDIAN_SI * PA_PER_MPA * np.exp(
        rs["upsilon"].standard_normal(n_p))
    state = (rs["state"].random(n_p) < slip_p).astype(np.int64)
    ang = rs["slipdir"].uniform(0.0, 2 * np.pi, n_p)
    q = rs["rhs"].standard_normal(n_p)
    aperture = None
    if open_p > 0:
        # Bernoulli(open_p) open faces (overriding slip), openings
        # U[0.5, 1.5] x APERTURE_REF
        state[rs["open"].random(n_p) < open_p] = 2
        aperture = APERTURE_REF * rs["open"].uniform(0.5, 1.5, n_p)
    s = build_system(shape, h, fr, E, ups, face_state=state, slip_angle=ang,
                     q=q, name=name, seed=seed, top_load=top_load,
                     aperture=aperture)
    s.extras["rng_obs"] = rs["obs"]
    s.extras["rng_rhs"] = rs["rhs"]
    return s


def tiny_system(shape=(3, 3, 3), fractures: Optional[List[Fracture]] = None,
                slip_p: float = 0.0, seed: int = 0, uniform_E: bool = False,
                name: str = "tiny", open_p: float = 0.0) -> BlockSystem:
    """A small system for exact / brute-force checks (unit cube)."""
    rs = _streams(seed)
    n = int(np.prod(shape))
    h = 1.0 / shape[0]
    if fractures is None:
        fractures = [Fracture(0, shape[0] // 2, 0, shape[1], 0, shape[2])]
    E = np.full(n, 1e4) if uniform_E else _lognormal_E(rs["E"], n)
    return _finish(name, shape, h, fractures, E, slip_p, rs, seed,
                   open_p=open_p)


def rhs_batch(s: BlockSystem, k: int = 32) -> np.ndarray:
    """``k`` right-hand sides with norms 10^(-2 + 4 i / (k-1)) (N x k).

    Column i is ``[f_i; 0; q_i]`` scaled to its norm, with ``f_i`` the top
    load times per-node N(1, 0.25^2) factors and ``q_i`` ~ N(0, I).
    """
    rng = np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([s.seed, 4242])))
    nn = s.n_u // 3
    base = s.b[:s.n_u]
    B = np.zeros((s.N, k))
    for i in range(k):
        fac = 1.0 + 0.25 * rng.standard_normal(nn)
        f = base * np.repeat(fac, 3)
        qv = rng.standard_normal(s.n_p)
        v = np.concatenate([f, np.zeros(s.n_t), qv])
        scale = 10.0 ** (-2.0 + 4.0 * i / max(k - 1, 1))
        B[:, i] = scale * v / np.linalg.norm(v)
    return B


def observations(s: BlockSystem, scale: float = 0.1) -> Tuple[np.ndarray, np.ndarray]:
    """``(xi, p_obs)``: p_obs is the fracture pressure at log-transmissibility
    ``log U + scale xi``.  With no open faces the pressure row of the system
    decouples, so ``p_obs = T(U e^(scale xi))^{-1} b_p`` exactly."""
    rng = s.extras.get("rng_obs")
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(s.seed + 7))
    xi = rng.standard_normal(s.n_p)
    if s.Q2.nnz:
        raise ValueError("observations assume decoupled pressure (Q2 = 0)")
    Tpert = assemble_T(s, s.upsilon * np.exp(scale * xi))
    bp = s.b[s.n_u + s.n_t:]
    p_obs = spla.spsolve(Tpert.tocsc(), bp)
    return xi, p_obs
