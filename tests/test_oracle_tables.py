"""Pins of the oracle's adaptive tables (Section II-B/C, Section III):
interpolation property, polynomial reproduction, the closed-form error bounds
of Eqs. (10)-(11), the hash of Eq. (6) against a brute-force search, the
forced zero samples, the merge rule, and the qualitative claims of the
interpolation experiment of Section IV-A."""

import numpy as np
import pytest

K2 = 2.0 * np.pi


def _b4(k, r):
    """|d^4/dr^4 (e^{-jkr}/r)| <= B4(r)/r (Leibniz)."""
    return k ** 4 + 4 * k ** 3 / r + 12 * k ** 2 / r ** 2 + 24 * k / r ** 3 + 24 / r ** 4


@pytest.fixture(scope="module")
def tabs(orc):
    out = {}
    for tol in (1e-4, 1e-6, 1e-8):
        out[("G", tol)] = orc.build_table(orc.GREEN, K2, 0.316, 1.98, tol)
        out[("E", tol)] = orc.build_table(orc.EXP, K2, 0.316, 1.98, tol)
    out[("G17", 1e-6)] = orc.build_table(orc.GREEN, 17.0, 0.0331, 1.9998, 1e-6)
    return out


def _exact(kind, k, r):
    e = np.exp(-1j * k * r)
    return e if kind == 0 else e / r


@pytest.mark.parametrize("key", [("G", 1e-4), ("G", 1e-8), ("E", 1e-6), ("G17", 1e-6)])
def test_interpolates_at_nodes(tabs, key):
    T = tabs[key]
    k = 17.0 if key[0] == "G17" else K2
    v = T(T.r)
    ex = _exact(T.kind, k, T.r)
    assert np.max(np.abs(v - ex) / np.abs(ex)) < 1e-14
    assert np.max(np.abs(T.f - ex) / np.abs(ex)) < 5e-16


def test_polynomial_reproduction(orc):
    rng = np.random.default_rng(7)
    r = np.sort(rng.uniform(0.5, 2.0, 300))
    r = r[np.concatenate([[True], np.diff(r) > 1e-3])]
    c = rng.standard_normal(8).view(np.complex128)
    cubic = lambda x: ((c[3] * x + c[2]) * x + c[1]) * x + c[0]  # noqa: E731
    affine = lambda x: c[1] * x + c[0]  # noqa: E731
    x = rng.uniform(r[0], r[-1], 5000)
    G = orc.table_from_nodes(orc.GREEN, r, cubic(r))
    assert np.max(np.abs(G(x) - cubic(x)) / np.abs(cubic(x))) < 1e-12
    E = orc.table_from_nodes(orc.EXP, r, affine(r))
    assert np.max(np.abs(E(x) - affine(x)) / np.abs(affine(x))) < 1e-13
    # a cubic is not reproduced by the linear rule (the check has teeth)
    E3 = orc.table_from_nodes(orc.EXP, r, cubic(r))
    assert np.max(np.abs(E3(x) - cubic(x))) > 1e-9


@pytest.mark.parametrize("tol", [1e-4, 1e-6, 1e-8])
def test_error_bounds_per_interval(tabs, tol):
    """Eq. (10) for the linear Exp table: |E - E_1| <= h^2 k^2/8 per interval;
    Eq. (11) for the cubic: |G - G_3| <= prod|r - r_j| max|G''''|/4!."""
    E = tabs[("E", tol)]
    h = np.diff(E.r)
    s = (np.arange(1, 9) / 9.0)[None, :]
    x = (E.r[:-1, None] + s * h[:, None]).ravel()
    err = np.abs(E(x) - _exact(0, K2, x)).reshape(-1, 8).max(1)
    assert np.all(err <= h ** 2 * K2 ** 2 / 8.0 * (1 + 1e-9) + 1e-15)
    G = tabs[("G", tol)]
    n = G.n
    x = (G.r[:-1, None] + s * np.diff(G.r)[:, None]).ravel()
    i = np.repeat(np.arange(n - 1), 8)
    st = np.clip(i - 1, 0, n - 4)
    om = np.ones_like(x)
    for j in range(4):
        om *= np.abs(x - G.r[st + j])
    lo = G.r[st]
    bound = om * (_b4(K2, lo) / lo) / 24.0
    err = np.abs(G(x) - _exact(1, K2, x))
    assert np.all(err <= bound * (1 + 1e-9) + 1e-15)


@pytest.mark.parametrize("key", [("G", 1e-4), ("G", 1e-6), ("G", 1e-8), ("E", 1e-4), ("E", 1e-6),
                                 ("E", 1e-8), ("G17", 1e-6)])
def test_probe_error_within_tol(tabs, key):
    T = tabs[key]
    tol = key[1]
    k = 17.0 if key[0] == "G17" else K2
    assert T.probe_err <= tol
    rng = np.random.default_rng(11)
    x = rng.uniform(T.r[0], T.r[-1], 20000)
    ex = _exact(T.kind, k, x)
    assert np.max(np.abs(T(x) - ex) / np.abs(ex)) <= tol


@pytest.mark.parametrize("key", [("G", 1e-4), ("G", 1e-8), ("E", 1e-6), ("G17", 1e-6)])
def test_hash_lookup_matches_search(tabs, key):
    T = tabs[key]
    rng = np.random.default_rng(5)
    r = T.r
    pts = [rng.uniform(r[0], r[-1], 20000), r, np.nextafter(r, 0), np.nextafter(r, 10)]
    b = np.arange(T.m) * T.delta + r[0]
    pts += [b[(b >= r[0]) & (b <= r[-1])], np.nextafter(b, 0)[(b > r[0]) & (b <= r[-1])]]
    x = np.concatenate(pts)
    x = x[(x >= r[0]) & (x <= r[-1])]
    ref = np.clip(np.searchsorted(r, x, side="right") - 1, 0, T.n - 2)
    got = np.array([T.lookup(v) for v in x])
    np.testing.assert_array_equal(got, ref)
    with pytest.raises(Exception):
        T.lookup(np.nextafter(r[0], 0))
    with pytest.raises(Exception):
        T.lookup(np.nextafter(r[-1], 10))


def test_hash_array_definition(tabs):
    """Every bucket holds the largest node index whose bucket is <= it."""
    for T in tabs.values():
        bkt = np.floor((T.r - T.r[0]) / T.delta).astype(np.int64)
        assert np.all(np.diff(bkt) >= 1)  # at most one node per bucket
        ref = np.searchsorted(bkt, np.arange(T.m), side="right") - 1
        np.testing.assert_array_equal(T.hash, ref)
        assert T.delta == np.min(np.diff(T.r))
        assert T.m == int(np.floor((T.r[-1] - T.r[0]) / T.delta)) + 1


@pytest.mark.parametrize("key", [("G", 1e-6), ("E", 1e-6), ("G17", 1e-6)])
def test_zeros_are_samples_and_merge_rule(tabs, key):
    T = tabs[key]
    k = 17.0 if key[0] == "G17" else K2
    c = np.pi / (2 * k)
    m = np.arange(int(np.floor(T.r[0] / c)) + 1, int(np.ceil(T.r[-1] / c)) + 1)
    z = m * c
    z = z[(z > T.r[0]) & (z < T.r[-1])]
    assert np.all(np.isin(z, T.r))  # forced zero samples, exactly
    gaps = np.diff(T.r)
    assert gaps.min() >= 0.25 * T.t * (1 - 1e-12)  # merge distance mu t
    assert gaps.max() <= 1.25 * T.t * (1 + 1e-12)
    # refined spacing t/2 around every zero
    for zz in z:
        i = np.searchsorted(T.r, zz)
        near = T.r[max(i - 2, 0): i + 3]
        near = near[np.abs(near - zz) <= T.t + 1e-15]
        assert np.allclose(np.diff(near), 0.5 * T.t, rtol=1e-9)


def _placement_by_definition(k, rmin, rmax, t, mu=0.25, half_window=2.0, ratio=0.5):
    """The sample positions of Section II-B written out plainly (readings:
    zeros of Re and Im at r = m pi / (2k) strictly inside the range; windows of
    half-width 2t about each zero sampled every t/2; uniform samples every t
    from r_min, dropped inside an open window; candidates visited as zeros,
    the two ends, refined samples, uniform samples, each kept only if it lies
    at least mu t from every sample kept before it).  A sorted list and
    bisection find the nearest kept sample; nothing is binned."""
    import bisect

    c = np.pi / (2.0 * k)
    m = np.arange(int(np.floor(rmin / c)) - 1, int(np.ceil(rmax / c)) + 2)
    zeros = [float(mm) * c for mm in m if rmin < float(mm) * c < rmax]
    nref = int(round(half_window / ratio))
    refined = [z + float(s) * (ratio * t) for z in zeros for s in range(-nref, nref + 1)
               if s != 0 and rmin < z + float(s) * (ratio * t) < rmax]
    uniform = []
    i = 0
    while rmin + float(i) * t < rmax:
        x = rmin + float(i) * t
        if not any(abs(x - z) < half_window * t for z in zeros):
            uniform.append(x)
        i += 1
    kept = []
    for x in zeros + [rmin, rmax] + refined + uniform:
        j = bisect.bisect_left(kept, x)
        near = [kept[jj] for jj in (j - 1, j) if 0 <= jj < len(kept)]
        if all(abs(x - y) >= mu * t for y in near):
            kept.insert(j, x)
    return np.array(kept)


@pytest.mark.parametrize("kind,k,rmin,rmax,tol", [
    (1, K2, 0.316, 1.98, 1e-4), (1, K2, 0.316, 1.98, 1e-8), (0, K2, 0.316, 1.98, 1e-6),
    (1, 17.0, 0.0331, 1.9998, 1e-5), (1, K2, 0.02977, 5.64474, 1e-6), (0, 10.0, 0.0, 2.0, 1e-6)])
def test_placement_matches_its_definition(orc, kind, k, rmin, rmax, tol):
    """The oracle's placement (a binned greedy merge) equals the plain
    definition sample for sample, at the spacing the probe check settled on."""
    T = orc.build_table(kind, k, rmin, rmax, tol)
    ref = _placement_by_definition(k, rmin, rmax, T.t)
    assert T.r.size == ref.size
    np.testing.assert_array_equal(T.r, ref)


def test_tables_reject_bad_arguments(orc):
    for args in [(0.0, 0.1, 1.0, 1e-6), (K2, 0.0, 1.0, 1e-6), (K2, 1.0, 0.5, 1e-6), (K2, 0.1, 1.0, 1.0)]:
        with pytest.raises(orc.OracleError):
            orc.build_table(orc.GREEN, *args)


def test_experiment_interpolation_accuracy(orc):
    """Section IV-A: r in [1e-4, 1] m, k = 2 pi, uniform interval t far from
    zeros, t/2 over a window of 4t around them, 1e4 test points, maximum
    relative error of the real and imaginary parts. The paper prints no
    values, so only its qualitative statements are checked: refinement helps
    the linear Exp table, and Lagrange beats linear for the Green function.
    Reading: t = lambda/1000 (Eq. (2)), random test points."""
    lam = 1.0
    t = lam / 1000.0
    rng = np.random.default_rng(12)
    x = np.sort(rng.uniform(1e-4, 1.0, 10000))

    def partwise(T, kind):
        ex = _exact(kind, K2, x)
        v = T(x)
        return (np.max(np.abs(v.real - ex.real) / np.abs(ex.real)),
                np.max(np.abs(v.imag - ex.imag) / np.abs(ex.imag)))

    e_plain = partwise(orc.build_table(orc.EXP, K2, 1e-4, 1.0, t=t, refine=False, zeros=False), 0)
    e_ref = partwise(orc.build_table(orc.EXP, K2, 1e-4, 1.0, t=t), 0)
    assert e_ref[0] < e_plain[0] and e_ref[1] < e_plain[1]
    # Green function away from the r_min singularity, linear vs Lagrange on
    # the same refined nodes
    G = orc.build_table(orc.GREEN, K2, 1e-4, 1.0, t=t)
    Gl = orc.table_from_nodes(orc.EXP, G.r, G.f)  # same nodes, linear rule
    far = x > 0.05
    ex = _exact(1, K2, x[far])
    assert np.max(np.abs(G(x[far]) - ex) / np.abs(ex)) < 1e-3 * np.max(np.abs(Gl(x[far]) - ex) / np.abs(ex))
