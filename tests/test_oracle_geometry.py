"""Pins of the oracle's geometry: quadrature, RWG topology, closed-form
potentials, ghat and the distance range. Each check compares with something
other than the oracle itself (closed forms, brute force, counting)."""

from math import factorial

import numpy as np
import pytest

from paper_1901_04162_amd import meshes


# ---- quadrature: exact on monomials up to the rule's degree ---------------

@pytest.mark.parametrize("q,deg", [(3, 2), (6, 4), (7, 5)])
def test_quadrature_exact_on_monomials(orc, q, deg):
    b, w = orc.quad_rule(q)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.all(b >= 0) and np.allclose(b.sum(1), 1.0, atol=1e-15)
    worst_above = 0.0
    for a0 in range(deg + 2):
        for a1 in range(deg + 2 - a0):
            for a2 in range(deg + 2 - a0 - a1):
                # mean of l0^a0 l1^a1 l2^a2 over the triangle
                exact = 2.0 * factorial(a0) * factorial(a1) * factorial(a2) / factorial(a0 + a1 + a2 + 2)
                got = np.sum(w * b[:, 0] ** a0 * b[:, 1] ** a1 * b[:, 2] ** a2)
                if a0 + a1 + a2 <= deg:
                    assert abs(got - exact) <= 2e-15, (a0, a1, a2)
                else:
                    worst_above = max(worst_above, abs(got - exact))
    assert worst_above > 1e-6  # the degree is not higher than claimed


# ---- RWG topology ---------------------------------------------------------

def _rwg_by_hand(F):
    """Independent construction with a dictionary (same numbering rule)."""
    seen = {}
    order = []
    for t, tri in enumerate(F):
        for a in range(3):
            u, v = int(tri[(a + 1) % 3]), int(tri[(a + 2) % 3])
            key = (min(u, v), max(u, v))
            if key not in seen:
                seen[key] = []
                order.append(key)
            seen[key].append((t, a, u == key[0]))
    out = []
    for key in order:
        h = seen[key]
        if len(h) != 2:
            continue
        plus = h[0] if h[0][2] else h[1]
        minus = h[1] if h[0][2] else h[0]
        out.append((key[0], key[1], plus[0], minus[0], plus[1], minus[1]))
    return np.array(out, dtype=np.int32)


@pytest.mark.parametrize("s", [0, 1, 2, 3])
def test_rwg_icosphere_counts_and_table(orc, s):
    V, F = meshes.icosphere(s)
    assert V.shape[0] == 10 * 4 ** s + 2 and F.shape[0] == 20 * 4 ** s
    E = orc.rwg(V, F)
    assert E.shape[0] == 30 * 4 ** s  # Euler: closed surface, every edge interior
    np.testing.assert_array_equal(E, _rwg_by_hand(F))
    for lo, hi, tp, tm, ap, am in E:
        assert {lo, hi} == set(F[tp]) - {F[tp][ap]}
        assert {lo, hi} == set(F[tm]) - {F[tm][am]}
        # T+ runs lo -> hi
        i = list(F[tp]).index(lo)
        assert F[tp][(i + 1) % 3] == hi


def test_rwg_plate_counts(orc):
    V, F = meshes.plate()
    assert V.shape == (10201, 3) and F.shape == (20000, 3)
    E = orc.rwg(V, F)
    assert E.shape[0] == 29800
    np.testing.assert_array_equal(E, _rwg_by_hand(F))


def test_rwg_rejects_bad_meshes(orc):
    V = np.zeros((5, 3))
    with pytest.raises(orc.OracleError):  # three triangles on one edge
        orc.rwg(V, np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4]]))
    with pytest.raises(orc.OracleError):  # inconsistent orientation
        orc.rwg(V, np.array([[0, 1, 2], [0, 1, 3]]))
    with pytest.raises(orc.OracleError):  # repeated vertex
        orc.rwg(V, np.array([[0, 0, 2]]))
    with pytest.raises(orc.OracleError):  # vertex out of range
        orc.rwg(V, np.array([[0, 1, 7]]))


# ---- closed-form potentials vs polar brute force -------------------------

def _composite_gauss(panels=200, n=60):
    g, gw = np.polynomial.legendre.leggauss(n)
    a = np.arange(panels)[:, None] / panels
    s = (a + 0.5 * (g[None, :] + 1.0) / panels).ravel()
    return s, np.tile(0.5 * gw / panels, panels)


def _polar_potentials(x, r):
    """S = int 1/R, V = int (r'-r)/R by polar integration about the projection
    of r, with the radial integral done exactly and composite Gauss-Legendre
    along each edge (a different derivation from the edge formulas of the
    oracle)."""
    x = [np.asarray(v, float) for v in x]
    nrm = np.cross(x[1] - x[0], x[2] - x[0])
    nrm /= np.linalg.norm(nrm)
    d = float(np.dot(nrm, r - x[0]))
    rho = r - d * nrm
    ad = abs(d)
    s, ws = _composite_gauss()
    S, Vv = 0.0, np.zeros(3)
    for i in range(3):
        a, b = x[i] - rho, x[(i + 1) % 3] - rho
        P = a[None, :] + s[:, None] * (b - a)[None, :]
        L = np.linalg.norm(P, axis=1)
        dth = np.dot(np.cross(P, (b - a)[None, :]), nrm) / L ** 2
        S += np.sum(ws * dth * (np.sqrt(L ** 2 + d * d) - ad))
        if ad > 0:
            rad = 0.5 * (L * np.sqrt(L ** 2 + d * d) - d * d * np.arcsinh(L / ad))
        else:
            rad = 0.5 * L ** 2
        Vv += np.sum((ws * dth * rad / L)[:, None] * P, axis=0)
    return S, Vv - d * nrm * S


_TRI = (np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.1, 0.0]), np.array([0.2, 0.9, 0.1]))


def _in_plane(u, v):
    x0, x1, x2 = _TRI
    return x0 + u * (x1 - x0) + v * (x2 - x0)


@pytest.mark.parametrize(
    "r",
    [
        _in_plane(0.3, 0.3),                       # inside, in plane
        _in_plane(0.3, 0.3) + [0.0, 0.0, 0.05],   # inside, just above
        _in_plane(0.5, 0.499),                     # near an edge
        _in_plane(0.001, 0.001),                   # near a vertex
        _in_plane(1.3, -0.2),                      # outside, in plane
        _in_plane(-0.5, 0.5),                      # on an edge line, outside
        np.array([0.5, 0.05, 0.3]),                # above
        np.array([2.0, 3.0, 1.0]),                 # far
    ],
)
def test_potentials_match_polar_integration(orc, r):
    S, V = orc.tri_potentials(*_TRI, r)
    S2, V2 = _polar_potentials(_TRI, r)
    assert abs(S - S2) <= 1e-12 * abs(S2)
    assert np.max(np.abs(V - V2)) <= 1e-12 * np.max(np.abs(V2))


def test_potentials_far_field(orc):
    x0, x1, x2 = _TRI
    A = 0.5 * np.linalg.norm(np.cross(x1 - x0, x2 - x0))
    c = (x0 + x1 + x2) / 3.0
    r = c + np.array([300.0, -200.0, 500.0])
    S, V = orc.tri_potentials(x0, x1, x2, r)
    D = np.linalg.norm(r - c)
    assert abs(S - A / D) < 1e-5 * A / D
    np.testing.assert_allclose(V, A * (c - r) / D, rtol=1e-5)


def test_ghat_limits(orc):
    k = 17.0
    assert orc.ghat(k, 0.0) == complex(0.0, -k)
    for R in [1e-9, 3e-6, 5.88e-6, 5.89e-6, 1e-4, 0.01, 0.3, 2.0]:
        ref = (np.exp(-1j * k * R) - 1.0) / R if R > 1e-3 else -1j * k - k * k * R / 2 + 1j * k ** 3 * R * R / 6 + k ** 4 * R ** 3 / 24
        assert abs(orc.ghat(k, R) - ref) <= 1e-9 * abs(ref)


# ---- distance range ------------------------------------------------------

def test_r_range_brute_force(orc):
    V, F = meshes.icosphere(1)
    b, w = orc.quad_rule(6)
    P = np.einsum("qc,tcx->tqx", b, V[F])  # quadrature points
    lo, hi = np.inf, 0.0
    for p in range(F.shape[0]):
        for q in range(F.shape[0]):
            if set(F[p]) & set(F[q]):
                continue
            D = np.linalg.norm(P[p][:, None, :] - P[q][None, :, :], axis=2)
            lo, hi = min(lo, D.min()), max(hi, D.max())
    rmin, rmax = orc.r_range(V, F, 6)
    assert abs(rmin - lo) <= 2e-16 * lo and abs(rmax - hi) <= 2e-16 * hi
