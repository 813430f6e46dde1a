"""Pins of the oracle's adjoint reference: the scalar loss L = Re sum conj(W) Z,
its vertex-local form, and its finite-difference gradient.

L is fixed by the matrix of Eq. (1)-(2) (EFIE Galerkin with RWG functions);
the gradient is pinned by what the mathematics of that matrix forces:
translation and rotation invariance, the homogeneity Z(aV, k/a) = a^2 Z(V, k)
(Euler: sum x.dL/dx - k dL/dk = 2L), and, for a pair of far-apart plates, a
closed-form d/dk of the quadrature sum written out here in numpy.
"""

import numpy as np
import pytest

from paper_1901_04162_amd import meshes

ETA0 = 376.730313668


def _small_mesh():
    V, F = meshes.icosphere(1)
    V = meshes.jitter_uniform(V, F, 0.08, 11)
    return V, F


def test_loss_is_weighted_sum_of_fill(orc):
    V, F = _small_mesh()
    edges = orc.rwg(V, F)
    k, Q = 3.0, 6
    W = meshes.dual_weights(edges.shape[0], 4)
    Z = orc.fill(V, F, k, Q, edges=edges)
    ref = float(np.real(np.sum(np.conj(W) * Z)))
    assert abs(orc.loss(V, F, edges, k, Q, W) - ref) <= 1e-12 * np.abs(W * Z).sum()


def test_local_loss_moves_like_full_loss(orc):
    """Only entries on triangles around a vertex change when it moves, so
    differences of the local loss equal differences of the full loss."""
    V, F = _small_mesh()
    edges = orc.rwg(V, F)
    k, Q = 3.0, 6
    W = meshes.dual_weights(edges.shape[0], 5)
    for v in (0, 17, 41):
        Vp = V.copy()
        Vp[v] += [0.013, -0.007, 0.021]
        d_full = orc.loss(Vp, F, edges, k, Q, W) - orc.loss(V, F, edges, k, Q, W)
        d_loc = orc.loss(Vp, F, edges, k, Q, W, v) - orc.loss(V, F, edges, k, Q, W, v)
        assert abs(d_full - d_loc) <= 1e-10 * max(1.0, abs(d_full))
        assert abs(d_full) > 1e-3


def test_fd_step_consistency(orc):
    """Richardson estimates at steps h and h/2 agree to O(h^4)."""
    V, F = _small_mesh()
    edges = orc.rwg(V, F)
    k, Q = 3.0, 6
    W = meshes.dual_weights(edges.shape[0], 6)
    idx = [0, 5, 31, 77, 100]
    g1, k1 = orc.grad_fd(V, F, edges, k, Q, W, idx, h=1e-4)
    g2, k2 = orc.grad_fd(V, F, edges, k, Q, W, idx, h=5e-5)
    scale = np.abs(g1).max()
    assert np.abs(g1 - g2).max() <= 1e-8 * scale
    assert abs(k1 - k2) <= 1e-8 * abs(k1)


@pytest.fixture(scope="module")
def full_grad(orc):
    V, F = _small_mesh()
    edges = orc.rwg(V, F)
    k, Q = 3.0, 6
    W = meshes.dual_weights(edges.shape[0], 7)
    g, gk = orc.grad_fd(V, F, edges, k, Q, W)
    L = orc.loss(V, F, edges, k, Q, W)
    return V, g.reshape(-1, 3), gk, L


def test_translation_invariance(full_grad):
    V, g, gk, L = full_grad
    assert np.abs(g.sum(0)).max() <= 1e-7 * np.abs(g).sum()


def test_rotation_invariance(full_grad):
    V, g, gk, L = full_grad
    torque = np.cross(V, g).sum(0)
    assert np.abs(torque).max() <= 1e-7 * (np.linalg.norm(V, axis=1)[:, None] * np.abs(g)).sum()


def test_scaling_homogeneity(full_grad):
    """Z(aV, k/a) = a^2 Z(V, k): every factor of Eq. (1) is a power of the
    length scale once kR is held fixed."""
    V, g, gk, L = full_grad
    k = 3.0
    lhs = float((V * g).sum()) - k * gk
    assert abs(lhs - 2 * L) <= 1e-7 * (np.abs(V * g).sum() + abs(k * gk) + abs(L))


def test_dk_closed_form_far_plates(orc):
    """d/dk of the regular quadrature sum between two far-apart two-triangle
    plates, written out in numpy: with c = j k eta/(4 pi) and
    B = (r - v).(r' - v')/4 - 1/k^2,
      dZ/dk = Z/k + c s s' l l' sum w w [ -j exp(-jkR) B + g 2/k^3 ]."""
    V = np.array([
        [0.0, 0.0, 0.0], [0.2, 0.0, 0.0], [0.0, 0.2, 0.0], [0.21, 0.19, 0.03],
        [1.5, 0.3, 0.4], [1.7, 0.3, 0.45], [1.5, 0.5, 0.4], [1.72, 0.52, 0.3],
    ])
    F = np.array([[0, 1, 2], [1, 3, 2], [4, 5, 6], [5, 7, 6]], dtype=np.int32)
    edges = orc.rwg(V, F)
    assert edges.shape[0] == 2
    k, Q = 4.0, 7
    b, w = orc.quad_rule(Q)
    W = np.array([[0.0, 0.7 - 0.2j], [-0.4 + 1.1j, 0.0]])

    def halves(e):
        vlo, vhi, tp, tm, ap, am = edges[e]
        l = np.linalg.norm(V[vlo] - V[vhi])
        return [(tp, F[tp][ap], 1.0, l), (tm, F[tm][am], -1.0, l)]

    def dz(m, n):
        c = 1j * k * ETA0 / (4 * np.pi)
        z = dzk = 0.0
        for t, va, s, l in halves(m):
            P = b @ V[F[t]]
            for u, vb, s2, l2 in halves(n):
                Qp = b @ V[F[u]]
                R = np.linalg.norm(P[:, None] - Qp[None], axis=2)
                E = np.exp(-1j * k * R)
                g = E / R
                B = 0.25 * ((P - V[va])[:, None, :] * (Qp - V[vb])[None]).sum(2) - 1 / k**2
                ww = np.outer(w, w)
                f = s * s2 * l * l2
                z += c * f * (ww * g * B).sum()
                dzk += c * f * (ww * (-1j * E * B + g * 2 / k**3)).sum()
        return z, z / k + dzk

    ref = sum(np.real(np.conj(W[m, n]) * dz(m, n)[1]) for m, n in ((0, 1), (1, 0)))
    zl = sum(np.real(np.conj(W[m, n]) * dz(m, n)[0]) for m, n in ((0, 1), (1, 0)))
    assert abs(orc.loss(V, F, edges, k, Q, W) - zl) <= 1e-12 * abs(zl)
    _, gk = orc.grad_fd(V, F, edges, k, Q, W, coords=[])
    assert abs(gk - ref) <= 1e-8 * abs(ref)
