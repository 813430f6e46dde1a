"""Pins of the oracle's MFIE operator (the magnetic-field integral equation
on the same RWG basis, Galerkin tested): the gradient of the triangle
potential against differences of the potential, the closed-form inner
integral of touching pairs against brute-force subdivided quadrature,
vanishing coplanar pairs, and, through the plane-wave solve, the sphere's
RCS against the Mie series."""

import numpy as np
import pytest

from oracle import scatter
from paper_1901_04162_amd import meshes

TRI = (np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.2]), np.array([0.3, 0.8, 0.0]))


@pytest.mark.parametrize("r", [[0.4, 0.3, 0.5], [1.5, -0.2, 0.1], [0.2, 0.2, -0.05],
                               [0.5, 0.05, 0.11], [0.0, 0.0, 0.3]])
def test_grad_potential_is_the_gradient(orc, r):
    r = np.array(r)
    g = orc.grad_potential(*TRI, r)
    h = 1e-5
    fd = np.zeros(3)
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        fd[c] = (orc.tri_potentials(*TRI, r + e)[0] - orc.tri_potentials(*TRI, r - e)[0]) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-8 * max(1.0, np.abs(g).max())


def test_grad_potential_far_field(orc):
    """Far away the triangle acts as a point charge of its area at the
    centroid: grad S -> -A d/|d|^3, with an O(|d|^-4) correction."""
    A = 0.5 * np.linalg.norm(np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0]))
    c = sum(TRI) / 3
    for u in ([0.3, 0.4, 0.866], [-1.0, 0.2, -0.3]):
        d = 1e3 * np.array(u) / np.linalg.norm(u)
        g = orc.grad_potential(*TRI, c + d)
        want = -A * d / np.linalg.norm(d) ** 3
        assert np.max(np.abs(g - want)) <= 1e-5 * np.abs(want).max()


def _subdivide(X, L):
    tris = [X]
    for _ in range(L):
        nxt = []
        for a, b, c in tris:
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            nxt += [np.array(t) for t in ([a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca])]
        tris = nxt
    return np.array(tris)


def _brute_block(orc, V, F, p, q, k, rule, L=5, n=8):
    """(1/4) sum_i w_i (1/A_q) int_q (r' - v_b).(t_i x d) K(R) dS' with the inner
    integral on 4^L sub-triangles, n x n collapsed Gauss points each."""
    b, w = rule
    bb, ww = orc.collapsed_gauss_rule(n)
    Xp, Xq = V[F[p]], V[F[q]]
    nrm = np.cross(Xp[1] - Xp[0], Xp[2] - Xp[0])
    nrm /= np.linalg.norm(nrm)
    T = _subdivide(Xq, L)
    P = np.einsum("qk,tkc->tqc", bb, T).reshape(-1, 3)
    At = 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1)
    W = (At[:, None] * ww[None, :]).ravel()
    Aq = 0.5 * np.linalg.norm(np.cross(Xq[1] - Xq[0], Xq[2] - Xq[0]))
    out = np.zeros((3, 3), complex)
    for i in range(len(w)):
        r = b[i] @ Xp
        d = r - P
        R = np.linalg.norm(d, axis=1)
        K = (1 + 1j * k * R) * np.exp(-1j * k * R) / R ** 3
        for a in range(3):
            td = np.cross(np.cross(r - Xp[a], nrm), d)
            for c in range(3):
                out[a, c] += w[i] * np.sum(W * np.einsum("pc,pc->p", P - Xq[c], td) * K) / Aq
    return 0.25 * out


# p = 0; q = 1 shares the edge (0, 1) at a fold; q = 2 shares vertex 1 only
_V = np.array([[0, 0, 0], [1, 0, 0], [0.3, 0.9, 0], [0.4, -0.5, 0.7], [1.8, 0.3, 0.5],
               [1.5, -0.6, -0.2], [4.0, 3.0, 2.0], [4.8, 3.1, 2.4], [4.2, 3.7, 1.9]], float)
_F = np.array([[0, 1, 2], [1, 0, 3], [1, 4, 5], [6, 7, 8]], np.int32)


@pytest.mark.parametrize("q", [1, 2])
@pytest.mark.parametrize("k,tol", [(0.5, 1e-6), (3.0, 1e-3)])
def test_touching_closed_form_matches_brute_force(orc, q, k, tol):
    """The closed-form inner integral (gradient of S, vector potential V and
    the k^2/2 term) plus the rule on the bounded remainder reproduce the
    brute-force inner integral; what is left is the rule's error on the
    remainder, which grows as k^3."""
    got = orc.mfie_pair_block(_V, _F, 0, q, k, 7)
    ref = _brute_block(orc, _V, _F, 0, q, k, orc.quad_rule(7))
    assert np.max(np.abs(got - ref)) <= tol * np.abs(ref).max()


def _symmetric_rule(orc, n):
    """Collapsed Gauss rule averaged over the three vertices."""
    b, w = orc.collapsed_gauss_rule(n)
    return (np.concatenate([b, b[:, [1, 2, 0]], b[:, [2, 0, 1]]]), np.concatenate([w, w, w]) / 3)


def test_vertex_touching_high_order(orc):
    rule = _symmetric_rule(orc, 6)
    got = orc.mfie_pair_block(_V, _F, 0, 2, 3.0, rule)
    ref = _brute_block(orc, _V, _F, 0, 2, 3.0, rule)
    assert np.max(np.abs(got - ref)) <= 1e-7 * np.abs(ref).max()


def test_far_pair_closed_form_equals_rule(orc):
    """On a distant pair the touching path (closed form + remainder) and the
    plain rule on K agree to the rule's accuracy."""
    for k in (0.7, 4.0):
        reg = orc.mfie_pair_block(_V, _F, 0, 3, k, 7)
        tch = orc.mfie_pair_block(_V, _F, 0, 3, k, 7, force_touching=True)
        assert np.max(np.abs(reg - tch)) <= 1e-6 * np.abs(reg).max()
    # with a rule fine enough for the oscillation, the rule on K equals the
    # brute-force inner integral
    rule = _symmetric_rule(orc, 8)
    reg = orc.mfie_pair_block(_V, _F, 0, 3, 4.0, rule)
    ref = _brute_block(orc, _V, _F, 0, 3, 4.0, rule, L=1, n=8)
    assert np.max(np.abs(reg - ref)) <= 1e-9 * np.abs(ref).max()


def test_coplanar_and_self_pairs_vanish(orc):
    """b.(t x d) = 0 when both triangles lie in one plane: t x d is then
    normal to the plane and b lies in it."""
    V = np.array([[0, 0, 0], [1, 0, 0], [0.3, 0.9, 0], [0.5, -0.8, 0], [2.5, 0.4, 0]], float)
    F = np.array([[0, 1, 2], [1, 0, 3], [1, 4, 2]], np.int32)
    for q in (0, 1, 2):
        blk = orc.mfie_pair_block(V, F, 0, q, 2.0, 7)
        assert np.abs(blk).max() <= 1e-14
        if q:
            blk = orc.mfie_pair_block(V, F, 0, q, 2.0, 7, force_touching=True)
            assert np.abs(blk).max() <= 1e-14


def test_static_mfie_rhs_is_closed_form(orc):
    """At k = 0 the excitation is (s l/2)(c - v).(n x H0) summed over the two
    triangles, for any rule exact on linear functions."""
    V, F = meshes.icosphere(1)
    V = meshes.jitter_uniform(V, F, 0.05, 3)
    E = orc.rwg(V, F)
    E0 = np.array([0.2, -1.0, 0.4 + 0.1j])
    kh = np.array([0.0, 0.6, 0.8])
    b, w = orc.quad_rule(3)
    got = scatter.rhs_planewave_mfie(V, F, E, 0.0, b, w, kh, E0)
    H0 = np.cross(kh, E0) / scatter.ETA0
    want = np.zeros(E.shape[0], complex)
    for e, (vlo, vhi, tp, tm, ap, am) in enumerate(E):
        l = np.linalg.norm(V[vlo] - V[vhi])
        for t, a, s in ((tp, ap, 1), (tm, am, -1)):
            X = V[F[t]]
            n = np.cross(X[1] - X[0], X[2] - X[0])
            n /= np.linalg.norm(n)
            want[e] += s * l / 2 * (X.mean(0) - X[a]) @ np.cross(n, H0)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def _solve_sphere(orc, s, k=1.0, Q=6):
    V, F = meshes.icosphere(s)
    E = orc.rwg(V, F)
    b, w = orc.quad_rule(Q)
    kh, E0 = np.array([0, 0, 1.0]), np.array([1.0, 0, 0])
    Im = np.linalg.solve(orc.mfie_fill(V, F, k, Q, edges=E),
                         scatter.rhs_planewave_mfie(V, F, E, k, b, w, kh, E0))
    Ie = np.linalg.solve(orc.fill(V, F, k, Q, edges=E),
                         scatter.rhs_planewave(V, F, E, k, b, w, kh, E0))
    th = np.linspace(0.0, np.pi, 37)
    dirs = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    sig = scatter.rcs(scatter.far_field(V, F, E, Im, k, b, w, dirs), dirs, k)
    ref = scatter.mie_rcs(k, 1.0, th, "E")
    return (float(np.linalg.norm(sig - ref) / np.linalg.norm(ref)),
            float(np.linalg.norm(Im - Ie) / np.linalg.norm(Ie)))


def test_mfie_sphere_rcs_converges_to_mie(orc):
    """Solved for a plane wave on the unit sphere at ka = 1, the MFIE gives
    the Mie E-plane RCS and the same current as the EFIE, both better on a
    finer mesh (a sign error in K, the identity term or the normal would
    leave an O(1) error)."""
    r2, c2 = _solve_sphere(orc, 2)
    r3, c3 = _solve_sphere(orc, 3)
    print("mfie rcs error vs Mie: ico2", r2, "ico3", r3, "current vs efie", c2, c3)
    assert r2 < 0.07 and r3 < 0.025 and r3 < 0.5 * r2
    assert c2 < 0.025 and c3 < 0.01 and c3 < 0.6 * c2


def test_table_mode_converges_to_direct(orc):
    """The MFIE kernel taken from the Green table, (1/R + jk) G(R)/R, tends
    to the direct kernel as the table tolerance tightens."""
    V, F = meshes.icosphere(1)
    V = meshes.jitter_uniform(V, F, 0.05, 5)
    E = orc.rwg(V, F)
    k, Q = 6.0, 6
    Zd = orc.mfie_fill(V, F, k, Q, edges=E)
    rmin, rmax = orc.r_range(V, F, Q)
    errs = []
    for tol in (1e-4, 1e-8):
        G = orc.build_table(orc.GREEN, k, rmin, rmax, tol)
        Zt = orc.mfie_fill(V, F, k, Q, edges=E, mode=orc.TABLE, gtable=G)
        errs.append(np.abs(Zt - Zd).max() / np.abs(Zd).max())
    assert errs[1] < 1e-8 and errs[1] < 1e-2 * errs[0]
