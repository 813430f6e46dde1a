"""Pins of the oracle's angular-transformation inner integrals (the paper's
own inner scheme, n points on each source edge) and of the EFIE fill built on
them: brute-force subdivided quadrature off and in the plane, the static
limit against the closed-form potentials, the Exp table from r = 0, the full
matrix against the singularity-cancellation fill under a common fine rule,
and the sphere's RCS against the Mie series."""

import numpy as np
import pytest

from oracle import scatter
from paper_1901_04162_amd import meshes

X = (np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.2]), np.array([0.3, 0.8, 0.0]))


def _subdivide(T, L):
    tris = [np.array(T)]
    for _ in range(L):
        nxt = []
        for a, b, c in tris:
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            nxt += [np.array(t) for t in ([a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca])]
        tris = nxt
    return np.array(tris)


def _points(orc, L=6, n=10):
    bb, ww = orc.collapsed_gauss_rule(n)
    T = _subdivide(X, L)
    P = np.einsum("qk,tkc->tqc", bb, T).reshape(-1, 3)
    A = 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1)
    return P, (A[:, None] * ww[None, :]).ravel()


def _plane(r):
    nrm = np.cross(X[1] - X[0], X[2] - X[0])
    nrm /= np.linalg.norm(nrm)
    h = nrm @ (r - X[0])
    return nrm, h, r - h * nrm


@pytest.mark.parametrize("r", [[0.4, 0.3, 0.5], [1.5, -0.2, 0.3], [0.5, 0.3, 0.05],
                               [2.5, 1.5, -0.1], [0.45, 0.3, -0.1]])
def test_inner_integrals_match_brute_force(orc, r):
    r = np.array(r)
    k = 3.0
    P, W = _points(orc)
    _, _, rho0 = _plane(r)
    R = np.linalg.norm(r - P, axis=1)
    G = np.exp(-1j * k * R) / R
    b0, b1 = np.sum(W * G), (W * G) @ (P - rho0)
    I0, I1 = orc.angular_inner(*X, r, k, 16)
    scale = abs(b0) * np.linalg.norm(X[1] - X[0])  # I1's natural size: I0 times a length
    assert abs(I0 - b0) <= 1e-9 * abs(b0)
    assert np.abs(I1 - b1).max() <= 1e-9 * scale
    # fewer points per edge: the edge rule converges spectrally
    e8 = abs(orc.angular_inner(*X, r, k, 8)[0] - b0) / abs(b0)
    e4 = abs(orc.angular_inner(*X, r, k, 4)[0] - b0) / abs(b0)
    assert e8 < 1e-6 and e8 < e4


@pytest.mark.parametrize("r", [[0.4, 0.3, 0.0], [0.4, 0.3, 0.2], [1.6, 0.9, 0.0],
                               [0.2, -0.4, -0.3]])
def test_static_limit_is_the_closed_form_potentials(orc, r):
    """k -> 0: with exp(-jkR)/R = 1/R - jk + O(k^2 R), I0 -> S - jkA and
    I1 -> int (r' - rho0)/R dS' - jk A (c - rho0) = V + h n S - jk A (c - rho0),
    from the closed-form potentials (in the plane and inside the triangle as
    well)."""
    r = np.array(r)
    k = 1e-5
    S, Vv = orc.tri_potentials(*X, r)
    nrm, h, rho0 = _plane(r)
    A = 0.5 * np.linalg.norm(np.cross(X[1] - X[0], X[2] - X[0]))
    c = sum(X) / 3
    I0, I1 = orc.angular_inner(*X, r, k, 16)
    assert abs(I0 - (S - 1j * k * A)) <= 1e-9 * abs(S)
    assert np.abs(I1 - (Vv + h * nrm * S - 1j * k * A * (c - rho0))).max() <= 1e-8 * abs(S)


def test_in_plane_singular_point(orc):
    """Observation point inside the source triangle (the self term): I0 and
    I1 equal the closed-form static parts plus the brute-force integral of
    the smooth remainder (exp(-jkR) - 1)/R."""
    r = np.array([0.4, 0.3, 0.0])
    _, h, rho0 = _plane(r)
    r = rho0  # exactly in the plane
    k = 4.0
    S, Vv = orc.tri_potentials(*X, r)
    P, W = _points(orc)
    R = np.linalg.norm(r - P, axis=1)
    rem = (np.exp(-1j * k * R) - 1.0) / R
    I0, I1 = orc.angular_inner(*X, r, k, 16)
    # the remainder has a kink at R = 0, so the subdivided rule itself is
    # good to about 1e-9 here
    assert abs(I0 - (S + np.sum(W * rem))) <= 3e-9 * abs(S)
    assert np.abs(I1 - (Vv + (W * rem) @ (P - rho0))).max() <= 3e-9 * abs(S)


def test_exp_table_from_the_origin(orc):
    """The Exp table may start at r = 0 (no singularity): exact at the
    samples, probe error within tol; the Green table may not."""
    k = 7.0
    T = orc.build_table(orc.EXP, k, 0.0, 2.0, 1e-6)
    assert T.r[0] == 0.0 and T.probe_err <= 1e-6
    v = T(np.array([0.0, T.r[5]]))
    assert abs(v[0] - 1.0) < 1e-15 and abs(v[1] - np.exp(-1j * k * T.r[5])) < 1e-15
    with pytest.raises(orc.OracleError):
        orc.build_table(orc.GREEN, k, 0.0, 2.0, 1e-6)


def test_rmax_is_the_largest_point_to_vertex_distance(orc):
    V, F = meshes.icosphere(1)
    V = meshes.jitter_uniform(V, F, 0.05, 4)
    b, w = orc.quad_rule(6)
    P = np.einsum("qk,tkc->tqc", b, V[F]).reshape(-1, 3)
    want = np.linalg.norm(P[:, None, :] - V[None, :, :], axis=2).max()
    assert orc.angular_rmax(V, F, 6) == want


def _symmetric_rule(orc, n):
    b, w = orc.collapsed_gauss_rule(n)
    return (np.concatenate([b, b[:, [1, 2, 0]], b[:, [2, 0, 1]]]), np.concatenate([w, w, w]) / 3)


def test_fill_agrees_with_singularity_cancellation(orc):
    """Under one common rule the angular-transformation fill (converged in n:
    12 and 16 points per edge agree, even for the collapsed rules' points
    next to the vertices) and the singularity-cancellation fill
    (the rule on both sides, closed-form 1/R part on touching pairs) approach
    each other as the rule is refined: what is left is the cancellation
    fill's rule error on its remainder, which has a kink at R = 0."""
    V, F = meshes.icosphere(0)
    V = meshes.jitter_uniform(V, F, 0.05, 3)
    E = orc.rwg(V, F)
    k = 2.0
    errs = []
    for nr in (5, 7, 10):
        rule = _symmetric_rule(orc, nr)
        Zr = orc.fill(V, F, k, rule, edges=E)
        Z12 = orc.angular_fill(V, F, k, rule, 12, edges=E)
        Z16 = orc.angular_fill(V, F, k, rule, 16, edges=E)
        assert np.abs(Z12 - Z16).max() <= 1e-6 * np.abs(Z16).max()
        errs.append(np.abs(Z16 - Zr).max() / np.abs(Zr).max())
    print("angular vs cancellation:", errs)
    assert errs[2] < 2e-4 and errs[2] < errs[1] < errs[0]


def test_table_mode_error_follows_tol(orc):
    V, F = meshes.icosphere(1)
    V = meshes.jitter_uniform(V, F, 0.05, 3)
    E = orc.rwg(V, F)
    k, Q = 3.0, 7
    rmax = orc.angular_rmax(V, F, Q)
    Zd = orc.angular_fill(V, F, k, Q, 8, edges=E)
    errs = []
    for tol in (1e-4, 1e-8):
        T = orc.build_table(orc.EXP, k, 0.0, rmax, tol)
        Zt = orc.angular_fill(V, F, k, Q, 8, edges=E, mode=orc.TABLE, etable=T)
        errs.append(np.abs(Zt - Zd).max() / np.abs(Zd).max())
    assert errs[0] < 1e-3 and errs[1] < 1e-7


def test_angular_sphere_rcs_converges_to_mie(orc):
    """The EFIE filled with angular-transformation inner integrals, solved on
    the unit sphere at ka = 1, gives the Mie E-plane RCS, better on the finer
    mesh (3.4 % and 0.86 %, as the singularity-cancellation fill)."""
    errs = []
    for s in (2, 3):
        V, F = meshes.icosphere(s)
        E = orc.rwg(V, F)
        k, Q = 1.0, 6
        b, w = orc.quad_rule(Q)
        Z = orc.angular_fill(V, F, k, Q, 6, edges=E)
        I = np.linalg.solve(Z, scatter.rhs_planewave(V, F, E, k, b, w, np.array([0, 0, 1.0]),
                                                     np.array([1.0, 0, 0])))
        th = np.linspace(0.0, np.pi, 37)
        d = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
        sig = scatter.rcs(scatter.far_field(V, F, E, I, k, b, w, d), d, k)
        ref = scatter.mie_rcs(k, 1.0, th, "E")
        errs.append(float(np.linalg.norm(sig - ref) / np.linalg.norm(ref)))
    print("angular rcs error vs Mie", errs)
    assert errs[0] < 0.05 and errs[1] < 0.015 and errs[1] < 0.5 * errs[0]
