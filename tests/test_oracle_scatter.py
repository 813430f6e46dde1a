"""Pins of the scattering reference (plane-wave excitation, far field, Mie
series of the PEC sphere) and, through it, of the oracle's EFIE matrix
against physics: the sphere's RCS from the oracle's Z must converge to the
Mie series as the mesh is refined."""

import numpy as np
import pytest

from oracle import scatter
from paper_1901_04162_amd import meshes


def test_mie_rayleigh_limit():
    # small sphere: backscatter 9 (ka)^4 pi a^2, total scattering (10/3)(ka)^4 pi a^2
    x = 0.01
    q_ext, q_sca, q_back = scatter.mie_cross_sections(x)
    assert abs(q_back / (9 * x ** 4) - 1) < 1e-3
    assert abs(q_sca / (10 / 3 * x ** 4) - 1) < 1e-3


@pytest.mark.parametrize("x", [0.5, 3.0, 12.0])
def test_mie_energy_and_symmetry(x):
    """A lossless sphere extinguishes what it scatters; the amplitudes agree
    forward (S1 = S2) and are opposite backward (S1 = -S2); the integrated
    bistatic cross-section equals the series for Q_sca."""
    q_ext, q_sca, q_back = scatter.mie_cross_sections(x)
    assert abs(q_ext - q_sca) <= 1e-10 * q_sca
    S1, S2 = scatter.mie_amplitudes(x, np.array([0.0, np.pi]))
    assert abs(S1[0] - S2[0]) <= 1e-12 * abs(S1[0])
    assert abs(S1[1] + S2[1]) <= 1e-12 * abs(S1[1])
    k, a = 1.0, x
    assert abs(4 * np.pi * abs(S1[1]) ** 2 / k ** 2 / (np.pi * a ** 2) - q_back) <= 1e-10 * q_back
    th, wt = np.polynomial.legendre.leggauss(200)
    th = 0.5 * np.pi * (th + 1)
    wt = 0.5 * np.pi * wt
    S1, S2 = scatter.mie_amplitudes(x, th)
    sca = np.pi / k ** 2 * np.sum(wt * (np.abs(S1) ** 2 + np.abs(S2) ** 2) * np.sin(th))
    assert abs(sca / (np.pi * a ** 2) - q_sca) <= 1e-8 * q_sca


def test_mie_optical_limit():
    # large sphere: backscatter approaches the geometric-optics pi a^2
    _, _, q_back = scatter.mie_cross_sections(150.0)
    assert abs(q_back - 1.0) < 0.05


def _small_mesh():
    V, F = meshes.icosphere(1)
    return meshes.jitter_uniform(V, F, 0.05, 3), F


def test_rhs_converges_to_high_order_rule(orc):
    V, F = _small_mesh()
    E = orc.rwg(V, F)
    k, khat, E0 = 2.5, np.array([0.3, -0.2, 0.93]), np.array([1.0, 0.5j, -0.2])
    khat = khat / np.linalg.norm(khat)
    b7, w7 = orc.quad_rule(7)
    bh, wh = orc.collapsed_gauss_rule(30)
    r7 = scatter.rhs_planewave(V, F, E, k, b7, w7, khat, E0)
    rh = scatter.rhs_planewave(V, F, E, k, bh, wh, khat, E0)
    bh2, wh2 = orc.collapsed_gauss_rule(40)
    rh2 = scatter.rhs_planewave(V, F, E, k, bh2, wh2, khat, E0)
    assert np.max(np.abs(rh - rh2)) <= 1e-12 * np.max(np.abs(rh))  # converged reference
    assert np.max(np.abs(r7 - rh)) <= 1e-4 * np.max(np.abs(rh))


def test_static_rhs_is_closed_form(orc):
    """At k = 0 the excitation is E0 . (s l/2)(c - v) summed over the two
    triangles, for any rule exact on linear functions."""
    V, F = _small_mesh()
    E = orc.rwg(V, F)
    E0 = np.array([0.2, -1.0, 0.4 + 0.1j])
    b, w = orc.quad_rule(3)
    got = scatter.rhs_planewave(V, F, E, 0.0, b, w, np.array([0, 0, 1.0]), E0)
    want = np.zeros(E.shape[0], complex)
    for e, (vlo, vhi, tp, tm, ap, am) in enumerate(E):
        l = np.linalg.norm(V[vlo] - V[vhi])
        for t, a, s in ((tp, ap, 1), (tm, am, -1)):
            c = V[F[t]].mean(0)
            want[e] += s * l / 2 * (c - V[F[t][a]]) @ E0
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_far_field_is_the_transposed_excitation(orc):
    """F(rhat).p = sum_n I_n V_n(khat = -rhat, E0 = p): the same integrals."""
    V, F = _small_mesh()
    E = orc.rwg(V, F)
    b, w = orc.quad_rule(6)
    rng = np.random.default_rng(2)
    I = rng.standard_normal(E.shape[0]) + 1j * rng.standard_normal(E.shape[0])
    d = np.array([[0.6, 0.0, 0.8], [0.0, -1.0, 0.0]])
    Ff = scatter.far_field(V, F, E, I, 1.7, b, w, d)
    for i in range(2):
        for p in np.eye(3):
            v = scatter.rhs_planewave(V, F, E, 1.7, b, w, -d[i], p)
            assert abs(Ff[i] @ p - I @ v) <= 1e-12 * np.abs(Ff[i]).max()


def _mom_rcs_error(orc, s, k=1.0, Q=6):
    V, F = meshes.icosphere(s)
    E = orc.rwg(V, F)
    Z = orc.fill(V, F, k, Q, edges=E)
    b, w = orc.quad_rule(Q)
    Vm = scatter.rhs_planewave(V, F, E, k, b, w, np.array([0, 0, 1.0]), np.array([1.0, 0, 0]))
    I = np.linalg.solve(Z, Vm)
    th = np.linspace(0.0, np.pi, 37)
    dirs = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)  # E-plane (phi = 0)
    sig = scatter.rcs(scatter.far_field(V, F, E, I, k, b, w, dirs), dirs, k)
    ref = scatter.mie_rcs(k, 1.0, th, "E")
    return float(np.linalg.norm(sig - ref) / np.linalg.norm(ref))


def test_oracle_sphere_rcs_converges_to_mie(orc):
    """The EFIE matrix of the oracle, solved for a plane wave on the unit
    sphere at ka = 1, reproduces the Mie E-plane RCS, better on a finer mesh
    (the faceted sphere is the main error)."""
    e2 = _mom_rcs_error(orc, 2)
    e3 = _mom_rcs_error(orc, 3)
    print("rcs error vs Mie: ico2", e2, "ico3", e3)
    assert e2 < 0.05 and e3 < 0.02 and e3 < 0.6 * e2
