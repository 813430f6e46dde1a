"""Host-side checks of libmomfill.so that need no GPU: it loads, exports every
function its header declares, and its mesh planning (RWG table, touching
pairs, error codes) agrees with the oracle."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1901_04162_amd import meshes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "momfill.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mf_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_1901_04162_amd as mf

    L = mf.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(mf._lib.EXPORTS)


@pytest.mark.parametrize("s", [1, 2, 3])
def test_rwg_table_matches_oracle(orc, s):
    import paper_1901_04162_amd as mf

    V, F = meshes.icosphere(s)
    m = mf.Mesh(F, V.shape[0])
    np.testing.assert_array_equal(m.edges(), orc.rwg(V, F))


def test_rwg_table_matches_oracle_plate(orc):
    import paper_1901_04162_amd as mf

    V, F = meshes.plate(n=20)
    m = mf.Mesh(F, V.shape[0])
    E = m.edges()
    np.testing.assert_array_equal(E, orc.rwg(V, F))
    assert m.n_edges == 3 * 20 * 20 - 2 * 20  # interior edges of an n x n split grid


def test_touching_pair_count():
    import paper_1901_04162_amd as mf

    V, F = meshes.icosphere(2)
    m = mf.Mesh(F, V.shape[0])
    ref = sum(1 for p in range(len(F)) for q in range(len(F)) if set(F[p]) & set(F[q]))
    assert m.n_touching() == ref


@pytest.mark.parametrize("F", [
    [[0, 1, 2], [1, 0, 3], [0, 1, 4]],   # edge on three triangles
    [[0, 1, 2], [0, 1, 3]],              # inconsistent orientation
    [[0, 0, 2], [0, 2, 3]],              # repeated vertex
    [[0, 1, 9], [1, 0, 3]],              # index out of range
    [[0, 1, 2]],                         # no interior edge
])
def test_mesh_errors(F):
    import paper_1901_04162_amd as mf

    with pytest.raises(mf.MomfillError) as e:
        mf.Mesh(np.array(F), 5)
    assert e.value.code == mf._lib.MF_EMESH


def test_argument_errors_without_gpu():
    import paper_1901_04162_amd as mf

    L = mf.lib()
    h = C.c_void_p()
    ws = C.c_void_p(1 << 20)  # never dereferenced: every call below fails its checks first
    assert L.mf_mesh_create(0, 1, None, C.byref(h)) == mf._lib.MF_EINVAL
    assert L.mf_build_tables(-1.0, 0.1, 1.0, 1e-6, ws, 1 << 20, C.byref(h), None) == mf._lib.MF_EINVAL
    assert L.mf_build_tables(1.0, 0.5, 0.1, 1e-6, ws, 1 << 20, C.byref(h), None) == mf._lib.MF_EINVAL
    assert L.mf_build_tables(1.0, 0.1, 1.0, 0.5, ws, 1 << 20, C.byref(h), None) == mf._lib.MF_EINVAL
    assert L.mf_build_tables(1.0, 0.1, 1.0, 1e-6, None, 1 << 20, C.byref(h), None) == mf._lib.MF_EINVAL
    assert L.mf_build_tables(1.0, 0.1, 1.0, 1e-6, C.c_void_p((1 << 20) + 8), 1 << 20, C.byref(h),
                             None) == mf._lib.MF_EINVAL
    V, F = meshes.icosphere(1)
    m = mf.Mesh(F, V.shape[0])
    z = C.c_void_p(1)
    assert L.mf_fill_Z(m.handle, z, 1.0, 5, 1, None, z, 0, m.n_edges, None) == mf._lib.MF_EINVAL
    assert L.mf_fill_Z(m.handle, z, -1.0, 3, 1, None, z, 0, m.n_edges, None) == mf._lib.MF_EINVAL
    assert L.mf_fill_Z(m.handle, z, 1.0, 3, 0, None, z, 0, m.n_edges, None) == mf._lib.MF_EINVAL
    assert L.mf_fill_Z(m.handle, z, 1.0, 3, 1, None, z, 0, m.n_edges - 1, None) == mf._lib.MF_EINVAL
    assert L.mf_fill_Z(m.handle, z, 1.0, 3, 7, None, z, 0, m.n_edges, None) == mf._lib.MF_EINVAL
    assert L.mf_fill_Z(m.handle, z, 1.0, 3, 1 | 0x30, None, z, 0, m.n_edges, None) == mf._lib.MF_EINVAL
    assert b"ldz" in L.mf_last_error() or L.mf_last_error()


def test_fill_choice_pinning_without_gpu():
    import paper_1901_04162_amd as mf

    V, F = meshes.icosphere(2)
    m = mf.Mesh(F, V.shape[0])
    for c in (-1, 0, 1, 2):
        m.set_fill_choice(c)
    for c in (-2, 3):
        with pytest.raises(mf.MomfillError) as e:
            m.set_fill_choice(c)
        assert e.value.code == mf._lib.MF_EINVAL
    assert mf.lib().mf_mesh_set_fill_choice(None, 0) == mf._lib.MF_EINVAL


@pytest.mark.parametrize("s", [2, 4])
def test_tile_plan_shape(s):
    import paper_1901_04162_amd as mf

    V, F = meshes.icosphere(s)
    m = mf.Mesh(F, V.shape[0])
    nb, nt, mt = m.plan()
    assert nt == nb * (nb + 1) // 2
    assert 1 <= mt <= 64
    assert nb * 80 >= m.n_edges


@pytest.mark.parametrize("s,r", [(2, 0.25), (3, 0.12)])
def test_near_pattern_brute_force(s, r):
    """The near-field CSR pattern equals a brute-force distance test on the
    edge midpoints (host planning only)."""
    import paper_1901_04162_amd as mf

    V, F = meshes.icosphere(s)
    m = mf.Mesh(F, V.shape[0])
    nf = mf.NearField(m, V, r)
    rp, col = nf.pattern()
    E = m.edges()
    mid = 0.5 * (V[E[:, 0]] + V[E[:, 1]])
    d2 = ((mid[:, None, :] - mid[None, :, :]) ** 2).sum(-1)
    near = d2 <= r * r
    assert nf.nnz == int(near.sum())
    for e in range(E.shape[0]):
        np.testing.assert_array_equal(col[rp[e]:rp[e + 1]], np.nonzero(near[e])[0])
    nb, nt, _ = m.plan()
    assert 1 <= nf.n_tiles <= nt


def test_workspaces_without_gpu():
    """The device memory model: sizes are queried, a mesh without a bound
    workspace refuses GPU work (no fallback allocation), a short or misaligned
    workspace is refused before anything touches it."""
    import paper_1901_04162_amd as mf

    L = mf.lib()
    V, F = meshes.icosphere(2)
    m = mf.Mesh(F, V.shape[0])
    n = C.c_size_t()
    assert L.mf_mesh_workspace_bytes(m.handle, C.byref(n)) == mf._lib.MF_OK
    # at least the 288-byte records and the FP64 quadrature points of every triangle
    assert n.value >= F.shape[0] * (288 + 3 * 7 * 8)
    fake = C.c_void_p(1 << 30)
    assert L.mf_mesh_set_workspace(m.handle, fake, n.value - 1, None) == mf._lib.MF_EINVAL
    assert b"too small" in L.mf_last_error()
    assert L.mf_mesh_set_workspace(m.handle, C.c_void_p((1 << 30) + 64), n.value, None) == \
        mf._lib.MF_EINVAL
    lo, hi = C.c_double(), C.c_double()
    assert L.mf_r_range(m.handle, fake, 3, C.byref(lo), C.byref(hi), None) == mf._lib.MF_EINVAL
    assert b"workspace" in L.mf_last_error()
    # table bounds grow as the tolerance tightens and cover the Exp table alone
    b = []
    for tol in (1e-4, 1e-6, 1e-8):
        t = C.c_size_t()
        assert L.mf_tables_workspace_bytes(17.0, 0.0331, 1.9998, tol, C.byref(t)) == mf._lib.MF_OK
        b.append(t.value)
    assert b[0] < b[1] < b[2]
    t = C.c_size_t()
    assert L.mf_exp_table_workspace_bytes(10.0, 2.0, 1e-6, C.byref(t)) == mf._lib.MF_OK
    assert t.value > 0
    arr = (C.c_void_p * 2)(m.handle.value, m.handle.value)
    assert L.mf_batch_workspace_bytes(2, arr, C.byref(t)) == mf._lib.MF_OK
    nf = mf.NearField(m, V, 0.2)
    assert L.mf_near_workspace_bytes(nf._h, C.byref(t)) == mf._lib.MF_OK and t.value > 0
