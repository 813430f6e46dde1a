"""Seeded synthetic inputs: triangle meshes, dual-weight matrices, entry samples.

This module holds input generators only (geometry and random numbers, no
electromagnetics). The paper's own sphere mesh and inductor geometry are not
published, so these stand in for them: icospheres for the PEC sphere of the
EFIE experiment (Section IV-B) and a jittered flat plate for a precision study.

Triangle order is hierarchical (icosphere: the four children of a face follow
each other; plate: cells in Morton order) so that consecutive triangles are
close in space. Every face is counter-clockwise seen from outside (icosphere)
or from +z (plate).
"""

from __future__ import annotations

import numpy as np

_PHI = (1.0 + 5.0 ** 0.5) / 2.0

_ICO_V = np.array(
    [
        (-1, _PHI, 0), (1, _PHI, 0), (-1, -_PHI, 0), (1, -_PHI, 0),
        (0, -1, _PHI), (0, 1, _PHI), (0, -1, -_PHI), (0, 1, -_PHI),
        (_PHI, 0, -1), (_PHI, 0, 1), (-_PHI, 0, -1), (-_PHI, 0, 1),
    ],
    dtype=np.float64,
)
_ICO_F = np.array(
    [
        (0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
        (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
        (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
        (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1),
    ],
    dtype=np.int32,
)


def icosphere(subdivisions: int, radius: float = 1.0):
    """Icosahedron subdivided `subdivisions` times (each face into four),
    midpoints pushed onto the sphere. Returns (V float64 [nv,3], F int32 [nt,3]).

    s = 2: 162 vertices, 320 triangles, 480 edges; s = 5: 10242 / 20480 / 30720.
    """
    V = [tuple(v / np.linalg.norm(v)) for v in _ICO_V]
    F = [tuple(int(i) for i in f) for f in _ICO_F]
    for _ in range(subdivisions):
        mid = {}

        def midpoint(a, b):
            key = (a, b) if a < b else (b, a)
            idx = mid.get(key)
            if idx is None:
                m = np.add(V[a], V[b]) * 0.5
                m = m / np.linalg.norm(m)
                idx = len(V)
                V.append(tuple(m))
                mid[key] = idx
            return idx

        G = []
        for a, b, c in F:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            G += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        F = G
    Vn = np.asarray(V, dtype=np.float64) * float(radius)
    Fn = np.asarray(F, dtype=np.int32)
    # outward orientation (the base faces above are listed counter-clockwise)
    c = Vn[Fn].mean(axis=1)
    n = np.cross(Vn[Fn[:, 1]] - Vn[Fn[:, 0]], Vn[Fn[:, 2]] - Vn[Fn[:, 0]])
    assert np.all(np.einsum("ij,ij->i", n, c) > 0.0)
    return Vn, Fn


def _morton_key(i: np.ndarray, j: np.ndarray) -> np.ndarray:
    key = np.zeros_like(i, dtype=np.int64)
    for bit in range(16):
        key |= ((i >> bit) & 1).astype(np.int64) << (2 * bit)
        key |= ((j >> bit) & 1).astype(np.int64) << (2 * bit + 1)
    return key


def plate(n: int = 100, h: float = 0.04, jitter: float = 0.002, seed: int = 3):
    """Flat plate of n x n square cells of side h in z = 0, each cell split into
    (a,b,c) and (a,c,d) with a=(i,j), b=(i+1,j), c=(i+1,j+1), d=(i,j+1);
    every vertex moved in x and y by U(-jitter, jitter) drawn from
    numpy.random.default_rng(seed). Cells are ordered along a Morton curve.
    Default: 10201 vertices, 20000 triangles, 29800 interior edges.
    """
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    V = np.zeros(((n + 1) * (n + 1), 3), dtype=np.float64)
    V[:, 0] = ii.ravel() * h
    V[:, 1] = jj.ravel() * h
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        V[:, :2] += rng.uniform(-jitter, jitter, size=(V.shape[0], 2))
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci, cj = ci.ravel(), cj.ravel()
    order = np.argsort(_morton_key(ci, cj), kind="stable")
    ci, cj = ci[order], cj[order]
    vid = lambda i, j: j * (n + 1) + i  # noqa: E731
    a, b, c, d = vid(ci, cj), vid(ci + 1, cj), vid(ci + 1, cj + 1), vid(ci, cj + 1)
    F = np.empty((2 * n * n, 3), dtype=np.int32)
    F[0::2] = np.stack([a, b, c], axis=1)
    F[1::2] = np.stack([a, c, d], axis=1)
    return V, F


def mean_edge_length(V: np.ndarray, F: np.ndarray) -> float:
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return float(np.linalg.norm(V[e[:, 0]] - V[e[:, 1]], axis=1).mean())


def jitter_uniform(V: np.ndarray, F: np.ndarray, frac: float, seed: int) -> np.ndarray:
    """Every coordinate moved by U(-frac, frac) x the mean edge length."""
    rng = np.random.default_rng(seed)
    return V + rng.uniform(-frac, frac, size=V.shape) * mean_edge_length(V, F)


def jitter_gauss(V: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """Every coordinate moved by N(0, sigma^2)."""
    rng = np.random.default_rng(seed)
    return V + rng.normal(0.0, sigma, size=V.shape)


def dual_weights(n_edges: int, seed: int) -> np.ndarray:
    """Complex n x n matrix with i.i.d. N(0,1) real and imaginary parts."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((n_edges, n_edges))
    im = rng.standard_normal((n_edges, n_edges))
    return (re + 1j * im).astype(np.complex128)


def entry_sample(n_edges: int, count: int, seed: int):
    """`count` distinct (row, col) pairs of an n_edges x n_edges matrix."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(n_edges * n_edges, size=count, replace=False)
    flat = np.sort(flat)
    return (flat // n_edges).astype(np.int64), (flat % n_edges).astype(np.int64)


# Named workloads: (description, mesh factory, k, quadrature points)
def workload(name: str):
    if name == "ico2":
        V, F = icosphere(2)
        return dict(V=V, F=F, k=2.0 * np.pi, Q=3)
    if name == "ico5":
        V, F = icosphere(5)
        return dict(V=V, F=F, k=17.0, Q=7)
    if name == "plate":
        V, F = plate()
        return dict(V=V, F=F, k=2.0 * np.pi, Q=7)
    if name == "ico4_grad":
        V, F = icosphere(4)
        V = jitter_gauss(V, 0.01, 5)
        return dict(V=V, F=F, k=10.0, Q=6)
    if name == "sweep":
        # three jittered icospheres (no re-projection) for a frequency sweep
        out = []
        for s, seed in ((3, 41), (4, 42), (5, 43)):
            V, F = icosphere(s)
            out.append((jitter_uniform(V, F, 0.05, seed), F))
        return dict(meshes=out, k=np.linspace(4.0, 20.0, 32), Q=6)
    raise KeyError(name)
