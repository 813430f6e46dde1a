"""Python access to the FP64 CPU oracle (liboracle.so, built from oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg import this module; the product package never does.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MOMFILL_ORACLE_SO names another build of oracle.c (the sanitizer test loads
# an ASan/UBSan build this way); default: the in-tree liboracle.so.
_SO_TREE = os.path.join(_HERE, "liboracle.so")
_SO = os.environ.get("MOMFILL_ORACLE_SO") or _SO_TREE

EXP, GREEN = 0, 1
TABLE, DIRECT = 0, 1
PART_ALL, PART_A, PART_PHI = 0, 1, 2
FORCE_TOUCHING = 4
ETA0 = 376.730313668


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, no FMA contraction, OpenMP)."""
    cmd = [
        "gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-Wall", "-Wextra",
        os.path.join(_HERE, "oracle.c"), "-o", _SO_TREE, "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return _SO_TREE


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        dp, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        vp = C.c_void_p
        L.or_quad_rule.argtypes = [C.c_int, dp, dp]
        L.or_rwg.argtypes = [C.c_int, C.c_int, ip, ip, ip]
        L.or_tri_potentials.argtypes = [dp, dp, dp, dp, dp, dp]
        L.or_tri_potentials.restype = None
        L.or_ghat.argtypes = [C.c_double, C.c_double, dp, dp]
        L.or_ghat.restype = None
        L.or_r_range.argtypes = [C.c_int, dp, C.c_int, ip, C.c_int, dp, dp, dp, dp]
        L.or_table_build.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.c_int, C.c_int, C.c_double, C.c_double,
                                     C.c_double, C.POINTER(vp)]
        L.or_table_from_nodes.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.POINTER(vp)]
        L.or_table_free.argtypes = [vp]
        L.or_table_free.restype = None
        L.or_table_info.argtypes = [vp, ip, ip, dp, dp, dp, ip]
        L.or_table_info.restype = None
        L.or_table_get.argtypes = [vp, dp, dp, ip]
        L.or_table_get.restype = None
        L.or_table_lookup.argtypes = [vp, C.c_double, ip]
        L.or_table_eval.argtypes = [vp, C.c_int, dp, dp]
        L.or_fill_entries.argtypes = [C.c_int, dp, C.c_int, ip, C.c_int, ip, C.c_double, C.c_int,
                                      dp, dp, C.c_int, C.c_int, vp, C.c_int64, lp, lp, dp]
        L.or_fill_rows.argtypes = [C.c_int, dp, C.c_int, ip, C.c_int, ip, C.c_double, C.c_int,
                                   dp, dp, C.c_int, C.c_int, vp, C.c_int, C.c_int, dp]
        L.or_pair_block.argtypes = [C.c_int, dp, C.c_int, ip, C.c_int, C.c_int, C.c_double,
                                    C.c_int, dp, dp, C.c_int, C.c_int, vp, dp]
        L.or_loss.argtypes = [C.c_int, dp, C.c_int, ip, C.c_int, ip, C.c_double, C.c_int, dp,
                              dp, dp, dp]
        L.or_loss_local.argtypes = [C.c_int, dp, C.c_int, ip, C.c_int, ip, C.c_double, C.c_int,
                                    dp, dp, dp, C.c_int, dp]
        L.or_max_threads.argtypes = []
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_threads.restype = None
        L.or_grad_potential.argtypes = [dp, dp, dp, dp, dp]
        L.or_grad_potential.restype = None
        L.or_mfie_pair_block.argtypes = [C.c_int, dp, C.c_int, ip, C.c_int, C.c_int, C.c_double,
                                         C.c_int, dp, dp, C.c_int, dp]
        L.or_angular_inner.argtypes = [dp, dp, dp, dp, C.c_double, C.c_int, C.c_int, vp, dp]
        L.or_angular_entries.argtypes = [C.c_int, dp, C.c_int, ip, C.c_int, ip, C.c_double,
                                         C.c_int, dp, dp, C.c_int, C.c_int, vp, C.c_int64, lp,
                                         lp, dp]
        L.or_angular_rmax.argtypes = [C.c_int, dp, C.c_int, ip, C.c_int, dp, dp, dp]
        L.or_mfie_entries.argtypes = [C.c_int, dp, C.c_int, ip, C.c_int, ip, C.c_double, C.c_int,
                                      dp, dp, C.c_int, vp, C.c_int64, lp, lp, dp]
        _lib = L
    return _lib


def max_threads() -> int:
    """Threads the oracle's OpenMP loops run on."""
    return int(lib().or_max_threads())


def set_threads(n: int) -> None:
    """Threads for the oracle's OpenMP loops from now on (timing runs)."""
    lib().or_set_threads(int(n))


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _pd(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _pi(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _pl(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def quad_rule(q: int):
    """(bary [q,3], w [q]) of the oracle's symmetric rule."""
    b = np.zeros((q, 3))
    w = np.zeros(q)
    if lib().or_quad_rule(q, _pd(b), _pd(w)) != q:
        raise OracleError(f"no {q}-point rule")
    return b, w


def _rule(Q):
    if isinstance(Q, tuple):
        b, w = Q
        return _d(b), _d(w)
    return quad_rule(int(Q))


def rwg(V, F):
    """Edges [E,6] int32: v_lo, v_hi, T+, T-, a+, a-."""
    F = _i(F)
    nt = F.shape[0]
    out = np.zeros((3 * nt // 2 + 1, 6), dtype=np.int32)
    ne = np.zeros(1, dtype=np.int32)
    _check(lib().or_rwg(int(np.asarray(V).shape[0]), nt, _pi(F), _pi(ne), _pi(out)), "rwg")
    return out[: int(ne[0])].copy()


def tri_potentials(x0, x1, x2, r):
    S = np.zeros(1)
    V = np.zeros(3)
    lib().or_tri_potentials(_pd(_d(x0)), _pd(_d(x1)), _pd(_d(x2)), _pd(_d(r)), _pd(S), _pd(V))
    return float(S[0]), V


def ghat(k, R):
    re, im = C.c_double(), C.c_double()
    lib().or_ghat(k, R, C.byref(re), C.byref(im))
    return complex(re.value, im.value)


def r_range(V, F, Q):
    V, F = _d(V), _i(F)
    b, w = _rule(Q)
    lo, hi = C.c_double(), C.c_double()
    _check(lib().or_r_range(V.shape[0], _pd(V), F.shape[0], _pi(F), len(w), _pd(b), _pd(w),
                            C.byref(lo), C.byref(hi)), "r_range")
    return lo.value, hi.value


class Table:
    """An oracle interpolation table (Exp: linear, Green: cubic Lagrange)."""

    def __init__(self, handle, kind):
        self._h = handle
        self.kind = kind
        n, m, it = C.c_int32(), C.c_int32(), C.c_int32()
        t, dl, pe = C.c_double(), C.c_double(), C.c_double()
        lib().or_table_info(handle, C.byref(n), C.byref(m), C.byref(t), C.byref(dl), C.byref(pe),
                            C.byref(it))
        self.n, self.m, self.t, self.delta = n.value, m.value, t.value, dl.value
        self.probe_err, self.iters = pe.value, it.value
        self.r = np.zeros(self.n)
        f = np.zeros(2 * self.n)
        self.hash = np.zeros(self.m, dtype=np.int32)
        lib().or_table_get(handle, _pd(self.r), _pd(f), _pi(self.hash))
        self.f = f[0::2] + 1j * f[1::2]

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_table_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def lookup(self, r: float) -> int:
        i = C.c_int32()
        _check(lib().or_table_lookup(self._h, float(r), C.byref(i)), "lookup")
        return i.value

    def __call__(self, r):
        r = _d(np.atleast_1d(r))
        out = np.zeros(2 * r.size)
        _check(lib().or_table_eval(self._h, r.size, _pd(r), _pd(out)), "table eval")
        return out[0::2] + 1j * out[1::2]


def build_table(kind, k, rmin, rmax, tol=1e-6, t=0.0, refine=True, zeros=True, mu=0.25, win=2.0,
                ratio=0.5) -> Table:
    h = C.c_void_p()
    _check(lib().or_table_build(kind, k, rmin, rmax, tol, t, int(refine), int(zeros), mu, win,
                                ratio, C.byref(h)), "table build")
    return Table(h, kind)


def table_from_nodes(kind, r, f) -> Table:
    r = _d(r)
    f = np.asarray(f, dtype=np.complex128)
    fre, fim = _d(f.real), _d(f.imag)
    h = C.c_void_p()
    _check(lib().or_table_from_nodes(kind, r.size, _pd(r), _pd(fre), _pd(fim), C.byref(h)),
           "table from nodes")
    return Table(h, kind)


def fill_entries(V, F, edges, k, Q, rows, cols, mode=DIRECT, part=PART_ALL, gtable=None):
    V, F, edges = _d(V), _i(F), _i(edges)
    b, w = _rule(Q)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros(2 * rows.size)
    _check(lib().or_fill_entries(V.shape[0], _pd(V), F.shape[0], _pi(F), edges.shape[0],
                                 _pi(edges), float(k), len(w), _pd(b), _pd(w), mode, part,
                                 gtable.handle if gtable is not None else None, rows.size,
                                 _pl(rows), _pl(cols), _pd(out)), "fill entries")
    return out[0::2] + 1j * out[1::2]


def fill_rows(V, F, edges, k, Q, r0, r1, mode=DIRECT, part=PART_ALL, gtable=None):
    """Rows [r0, r1) of Z in triangle-pair order (each pair's kernel values
    once for its nine local entries): the CPU baseline of the fill."""
    V, F, edges = _d(V), _i(F), _i(edges)
    b, w = _rule(Q)
    ne = edges.shape[0]
    out = np.zeros(2 * (r1 - r0) * ne)
    _check(lib().or_fill_rows(V.shape[0], _pd(V), F.shape[0], _pi(F), ne, _pi(edges), float(k),
                              len(w), _pd(b), _pd(w), mode, part,
                              gtable.handle if gtable is not None else None, int(r0), int(r1),
                              _pd(out)), "fill rows")
    return (out[0::2] + 1j * out[1::2]).reshape(r1 - r0, ne)


def fill(V, F, k, Q, mode=DIRECT, part=PART_ALL, gtable=None, edges=None):
    """Full E x E matrix, one entry at a time."""
    if edges is None:
        edges = rwg(V, F)
    E = edges.shape[0]
    rr, cc = np.meshgrid(np.arange(E), np.arange(E), indexing="ij")
    z = fill_entries(V, F, edges, k, Q, rr.ravel(), cc.ravel(), mode, part, gtable)
    return z.reshape(E, E)


def pair_block(V, F, p, q, k, Q, mode=DIRECT, part=PART_ALL, gtable=None):
    V, F = _d(V), _i(F)
    b, w = _rule(Q)
    out = np.zeros(18)
    _check(lib().or_pair_block(V.shape[0], _pd(V), F.shape[0], _pi(F), p, q, float(k), len(w),
                               _pd(b), _pd(w), mode, part,
                               gtable.handle if gtable is not None else None, _pd(out)),
           "pair block")
    return (out[0::2] + 1j * out[1::2]).reshape(3, 3)


def collapsed_gauss_rule(n: int):
    """n*n-point rule on the triangle from Gauss-Legendre on the square,
    collapsed at vertex 0 (weights sum to one). For convergence tests."""
    x, wx = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1.0)
    wx = 0.5 * wx
    u, v = np.meshgrid(x, x, indexing="ij")
    wu, wv = np.meshgrid(wx, wx, indexing="ij")
    l1 = u * (1.0 - v)
    l2 = u * v
    l0 = 1.0 - l1 - l2
    w = 2.0 * wu * wv * u
    b = np.stack([l0.ravel(), l1.ravel(), l2.ravel()], axis=1)
    return b, w.ravel()


def loss(V, F, edges, k, Q, W, vertex=None):
    """L = Re sum conj(W) Z (direct mode); with `vertex`, only the entries that
    move with that vertex (so differences in it equal differences of L)."""
    V, F, edges = _d(V), _i(F), _i(edges)
    b, w = _rule(Q)
    Wd = np.ascontiguousarray(np.asarray(W, dtype=np.complex128)).view(np.float64)
    out = C.c_double()
    args = [V.shape[0], _pd(V), F.shape[0], _pi(F), edges.shape[0], _pi(edges), float(k), len(w),
            _pd(b), _pd(w), _pd(Wd)]
    if vertex is None:
        _check(lib().or_loss(*args, C.byref(out)), "loss")
    else:
        _check(lib().or_loss_local(*args, int(vertex), C.byref(out)), "loss")
    return out.value


def grad_fd(V, F, edges, k, Q, W, coords=None, with_k=True, h=1e-4):
    """Gradient of L by central differences with one Richardson step
    (steps h and h/2, error O(h^4)): dL/dV at the given flat coordinate
    indices (all if None) and dL/dk.  This is the derivative by its
    definition, evaluated on the FP64 oracle."""
    V = np.array(V, dtype=np.float64)
    n = V.size
    idx = np.arange(n) if coords is None else np.asarray(coords)
    g = np.zeros(len(idx))
    for s, c in enumerate(idx):
        v = int(c) // 3
        d = []
        for hh in (h, h / 2):
            Vp = V.copy()
            Vp.flat[c] += hh
            Vm = V.copy()
            Vm.flat[c] -= hh
            d.append((loss(Vp, F, edges, k, Q, W, v) - loss(Vm, F, edges, k, Q, W, v)) / (2 * hh))
        g[s] = (4 * d[1] - d[0]) / 3
    gk = None
    if with_k:
        hk = h * k
        d = [(loss(V, F, edges, k + hh, Q, W) - loss(V, F, edges, k - hh, Q, W)) / (2 * hh)
             for hh in (hk, hk / 2)]
        gk = (4 * d[1] - d[0]) / 3
    return g, gk


def grad_potential(x0, x1, x2, r):
    """Gradient of S(r) = int dS'/|r - r'| over the triangle (x0, x1, x2)."""
    a = [np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in (x0, x1, x2, r)]
    g = np.zeros(3)
    lib().or_grad_potential(*[_pd(v) for v in a], _pd(g))
    return g


def mfie_pair_block(V, F, p, q, k, Q, force_touching=False):
    """3x3 block of the MFIE K operator for triangles p (test) and q."""
    V, F = _d(V), _i(F)
    b, w = _rule(Q)
    out = np.zeros(18)
    _check(lib().or_mfie_pair_block(V.shape[0], _pd(V), F.shape[0], _pi(F), int(p), int(q),
                                    float(k), len(w), _pd(b), _pd(w), int(force_touching),
                                    _pd(out)), "mfie pair block")
    return (out[0::2] + 1j * out[1::2]).reshape(3, 3)


def mfie_entries(V, F, edges, k, Q, rows, cols, mode=DIRECT, gtable=None):
    """MFIE matrix entries <f_m, f_n>/2 - K_mn (FP64); regular pairs take the
    kernel from the direct exponential or (mode=TABLE) from the Green table."""
    V, F, edges = _d(V), _i(F), _i(edges)
    b, w = _rule(Q)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros(2 * rows.size)
    _check(lib().or_mfie_entries(V.shape[0], _pd(V), F.shape[0], _pi(F), edges.shape[0],
                                 _pi(edges), float(k), len(w), _pd(b), _pd(w), int(mode),
                                 gtable.handle if gtable is not None else None, rows.size,
                                 _pl(rows), _pl(cols), _pd(out)), "mfie entries")
    return out[0::2] + 1j * out[1::2]


def mfie_fill(V, F, k, Q, edges=None, mode=DIRECT, gtable=None):
    """Full MFIE matrix, one entry at a time."""
    if edges is None:
        edges = rwg(V, F)
    E = edges.shape[0]
    rr, cc = np.meshgrid(np.arange(E), np.arange(E), indexing="ij")
    return mfie_entries(V, F, edges, k, Q, rr.ravel(), cc.ravel(), mode, gtable).reshape(E, E)


def angular_inner(x0, x1, x2, r, k, n, mode=DIRECT, etable=None):
    """(I0, I1): int_q exp(-jkR)/R dS' and int_q (r' - rho0) exp(-jkR)/R dS' by
    the angular transformation with n points per edge."""
    out = np.zeros(8)
    a = [np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in (x0, x1, x2, r)]
    _check(lib().or_angular_inner(*[_pd(v) for v in a], float(k), int(n), int(mode),
                                  etable.handle if etable is not None else None, _pd(out)),
           "angular inner")
    return complex(out[0], out[1]), out[2::2] + 1j * out[3::2]


def angular_entries(V, F, edges, k, Q, n_edge, rows, cols, mode=DIRECT, etable=None):
    """EFIE entries with every inner integral by the angular transformation."""
    V, F, edges = _d(V), _i(F), _i(edges)
    b, w = _rule(Q)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros(2 * rows.size)
    _check(lib().or_angular_entries(V.shape[0], _pd(V), F.shape[0], _pi(F), edges.shape[0],
                                    _pi(edges), float(k), len(w), _pd(b), _pd(w), int(n_edge),
                                    int(mode), etable.handle if etable is not None else None,
                                    rows.size, _pl(rows), _pl(cols), _pd(out)), "angular entries")
    return out[0::2] + 1j * out[1::2]


def angular_fill(V, F, k, Q, n_edge, edges=None, mode=DIRECT, etable=None):
    if edges is None:
        edges = rwg(V, F)
    E = edges.shape[0]
    rr, cc = np.meshgrid(np.arange(E), np.arange(E), indexing="ij")
    return angular_entries(V, F, edges, k, Q, n_edge, rr.ravel(), cc.ravel(), mode,
                           etable).reshape(E, E)


def angular_rmax(V, F, Q):
    V, F = _d(V), _i(F)
    b, w = _rule(Q)
    out = C.c_double()
    _check(lib().or_angular_rmax(V.shape[0], _pd(V), F.shape[0], _pi(F), len(w), _pd(b), _pd(w),
                                 C.byref(out)), "angular rmax")
    return out.value
