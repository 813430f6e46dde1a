"""FP64 reference for plane-wave scattering from a PEC body with the EFIE
(Section IV-B: the PEC sphere under an x-polarised plane wave along z).

TEST INFRASTRUCTURE ONLY: used by the tests and never by the product path.
Plain numpy, one basis function at a time.

Conventions are those of the fill: time factor exp(+j omega t), fields
exp(-j k khat.r), RWG functions f = s l/(2A) (r - v) on the two triangles of
each interior edge, eta0 = 376.730313668.

  excitation  V_m = int f_m . E_inc dS = sum_tri s l/2 sum_i w_i (r_i - v) . E0 exp(-j k khat.r_i)
  far field   F(rhat) = sum_n I_n int f_n exp(+j k rhat.r') dS'
              E_far = -j k eta0 exp(-jkr)/(4 pi r) (F - rhat (rhat.F))
  RCS         sigma = 4 pi r^2 |E_far|^2 / |E0|^2 = (k eta0)^2/(4 pi) |F_t|^2 / |E0|^2

The Mie series for a perfectly conducting sphere follows Bohren and Huffman
(Absorption and Scattering of Light by Small Particles, 1983, Sections 4.4
and 4.8) in the limit of infinite refractive index:
  a_n = [x j_n(x)]' / [x h_n(x)]',   b_n = j_n(x) / h_n(x),   h_n = j_n + i y_n,
  S1 = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n),
  S2 = sum (2n+1)/(n(n+1)) (a_n tau_n + b_n pi_n),
with sigma = 4 pi |S2|^2/k^2 in the E-plane (phi = 0, theta-polarised
scattered field) and 4 pi |S1|^2/k^2 in the H-plane (phi = 90 deg).  Only
|S|^2 enters the cross-sections, so the time convention drops out.
"""

from __future__ import annotations

import numpy as np
from scipy import special

ETA0 = 376.730313668


def _halves(V, F, edges):
    """Per edge: the two (triangle, free vertex, sign) and the edge length."""
    out = []
    for e in range(edges.shape[0]):
        vlo, vhi, tp, tm, ap, am = (int(x) for x in edges[e])
        l = float(np.linalg.norm(V[vlo] - V[vhi]))
        out.append(((tp, F[tp][ap], 1.0), (tm, F[tm][am], -1.0), l))
    return out


def rhs_planewave(V, F, edges, k, bary, w, khat, E0):
    """V_m = int f_m . E0 exp(-j k khat.r) dS with the triangle rule (bary, w)."""
    V = np.asarray(V, dtype=np.float64)
    khat = np.asarray(khat, dtype=np.float64)
    E0 = np.asarray(E0, dtype=np.complex128)
    out = np.zeros(edges.shape[0], dtype=np.complex128)
    for e, (hp, hm, l) in enumerate(_halves(V, F, edges)):
        acc = 0.0j
        for t, v, s in (hp, hm):
            P = bary @ V[F[t]]
            ph = np.exp(-1j * k * (P @ khat))
            acc += s * l / 2.0 * np.sum(w * ph * ((P - V[v]) @ E0))
        out[e] = acc
    return out


def rhs_planewave_mfie(V, F, edges, k, bary, w, khat, E0):
    """V_m = int f_m . (n x H_inc) dS, H_inc = khat x E0 exp(-j k khat.r)/eta0,
    n the outward unit normal of each (counter-clockwise) triangle."""
    V = np.asarray(V, dtype=np.float64)
    khat = np.asarray(khat, dtype=np.float64)
    H0 = np.cross(khat, np.asarray(E0, dtype=np.complex128)) / ETA0
    out = np.zeros(edges.shape[0], dtype=np.complex128)
    for e, (hp, hm, l) in enumerate(_halves(V, F, edges)):
        acc = 0.0j
        for t, v, s in (hp, hm):
            X = V[F[t]]
            n = np.cross(X[1] - X[0], X[2] - X[0])
            n /= np.linalg.norm(n)
            P = bary @ X
            ph = np.exp(-1j * k * (P @ khat))
            acc += s * l / 2.0 * np.sum(w * ph * ((P - V[v]) @ np.cross(n, H0)))
        out[e] = acc
    return out


def far_field(V, F, edges, I, k, bary, w, dirs):
    """F(rhat) = sum_n I_n int f_n exp(+j k rhat.r') dS' for each unit rhat."""
    V = np.asarray(V, dtype=np.float64)
    dirs = np.asarray(dirs, dtype=np.float64)
    out = np.zeros((dirs.shape[0], 3), dtype=np.complex128)
    for e, (hp, hm, l) in enumerate(_halves(V, F, edges)):
        for t, v, s in (hp, hm):
            P = bary @ V[F[t]]
            ph = np.exp(1j * k * (dirs @ P.T))          # [ndir, Q]
            out += I[e] * s * l / 2.0 * (ph * w) @ (P - V[v])
    return out


def rcs(Ffar, dirs, k, E0_norm=1.0):
    """Bistatic RCS from the far-field vectors of far_field()."""
    dirs = np.asarray(dirs, dtype=np.float64)
    Ft = Ffar - dirs * np.sum(dirs * Ffar, axis=1, keepdims=True)
    return (k * ETA0) ** 2 / (4 * np.pi) * np.sum(np.abs(Ft) ** 2, axis=1) / E0_norm ** 2


def mie_coefficients(x, nmax=None):
    """a_n, b_n (n = 1..nmax) of a perfectly conducting sphere, size x = k a."""
    if nmax is None:
        nmax = int(np.ceil(x + 4.05 * x ** (1.0 / 3.0) + 2))
    n = np.arange(1, nmax + 1)
    jn = special.spherical_jn(n, x)
    jnp = special.spherical_jn(n, x, derivative=True)
    yn = special.spherical_yn(n, x)
    ynp = special.spherical_yn(n, x, derivative=True)
    hn = jn + 1j * yn
    hnp = jnp + 1j * ynp
    # [x z_n(x)]' = z_n(x) + x z_n'(x)
    a = (jn + x * jnp) / (hn + x * hnp)
    b = jn / hn
    return n, a, b


def _pi_tau(n, mu):
    """Angular functions pi_n, tau_n at cos(theta) = mu (Bohren and Huffman 4.47)."""
    nmax = n[-1]
    pi = np.zeros((nmax + 1,) + np.shape(mu))
    tau = np.zeros_like(pi)
    pi[1] = 1.0
    tau[1] = mu
    for m in range(2, nmax + 1):
        p0 = pi[m - 2] if m >= 2 else 0.0
        pi[m] = (2 * m - 1) / (m - 1) * mu * pi[m - 1] - m / (m - 1) * p0
        tau[m] = m * mu * pi[m] - (m + 1) * pi[m - 1]
    return pi[1:], tau[1:]


def mie_amplitudes(x, theta):
    """S1(theta), S2(theta) of the perfectly conducting sphere."""
    n, a, b = mie_coefficients(x)
    mu = np.cos(np.asarray(theta, dtype=np.float64))
    pi, tau = _pi_tau(n, mu)
    c = ((2 * n + 1) / (n * (n + 1)))[:, None]
    pi, tau = pi.reshape(len(n), -1), tau.reshape(len(n), -1)
    S1 = np.sum(c * (a[:, None] * pi + b[:, None] * tau), axis=0)
    S2 = np.sum(c * (a[:, None] * tau + b[:, None] * pi), axis=0)
    return S1.reshape(np.shape(theta)), S2.reshape(np.shape(theta))


def mie_rcs(k, a, theta, plane="E"):
    """Bistatic RCS (m^2) of a PEC sphere of radius a at angle theta from the
    forward direction, in the E-plane (phi = 0) or the H-plane (phi = 90 deg)."""
    S1, S2 = mie_amplitudes(k * a, theta)
    S = S2 if plane == "E" else S1
    return 4 * np.pi * np.abs(S) ** 2 / k ** 2


def mie_cross_sections(x):
    """(Q_ext, Q_sca, Q_back) efficiencies (cross-section / (pi a^2))."""
    n, a, b = mie_coefficients(x)
    q_ext = 2.0 / x ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    q_sca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    q_back = 1.0 / x ** 2 * np.abs(np.sum((2 * n + 1) * (-1.0) ** n * (a - b))) ** 2
    return q_ext, q_sca, q_back
