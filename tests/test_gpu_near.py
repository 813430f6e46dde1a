"""GPU parity of the near-field fill (Section II-A): the CSR values must be
the entries the dense fill computes at the pattern's positions (same
kernels, same arithmetic) and agree with the oracle's entries."""

import sys

import numpy as np
import pytest

from paper_1901_04162_amd import meshes

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mf():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1901_04162_amd as m

    m.lib()
    return m


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _coo(rp, col):
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return rows.astype(np.int64), col.astype(np.int64)


@pytest.mark.parametrize("mode,dtype", [("table", "c64"), ("direct", "c128")])
def test_near_small_against_dense_and_oracle(mf, orc, mode, dtype):
    import torch

    V, F = meshes.icosphere(2)
    k, Q, r = 2 * np.pi, 3, 0.3
    say("near ico2", mode, dtype)
    m = mf.Mesh(F, V.shape[0])
    nf = mf.NearField(m, V, r)
    rows, cols = _coo(*nf.pattern())
    T = None
    if mode == "table":
        lo, hi = mf.r_range(m, V, Q)
        T = mf.build_tables(k, lo, hi, 1e-8)
    dt = torch.complex64 if dtype == "c64" else torch.complex128
    vals = nf.fill(V, k, Q, mode, T, dtype=dt).cpu().numpy()
    Z = mf.fill_Z(m, V, k, Q, mode, T, dtype=dt).cpu().numpy()
    mf.sync_status(m)
    e_dense = _rel(vals, Z[rows, cols])
    ref = orc.fill_entries(V, F, m.edges(), k, Q, rows, cols)
    e_orc = _rel(vals, ref)
    say(f"  nnz {nf.nnz} tiles {nf.n_tiles}: vs dense {e_dense:.2e}, vs oracle {e_orc:.2e}")
    assert e_dense <= 1e-6
    assert e_orc <= (1e-6 if mode == "direct" else 1e-5)


def test_near_self_only(mf):
    """A radius below the shortest midpoint distance leaves the diagonal."""
    import torch

    V, F = meshes.icosphere(1)
    m = mf.Mesh(F, V.shape[0])
    nf = mf.NearField(m, V, 1e-6)
    assert nf.nnz == m.n_edges
    rows, cols = _coo(*nf.pattern())
    assert np.array_equal(rows, cols)
    vals = nf.fill(V, 3.0, 6, "direct", dtype=torch.complex128).cpu().numpy()
    Z = mf.fill_Z(m, V, 3.0, 6, "direct", dtype=torch.complex128).cpu().numpy()
    assert _rel(vals, np.diag(Z)) <= 1e-6


def test_near_full_size(mf, orc):
    """The 30,720-unknown icosphere at k = 17 with a quarter-wavelength
    radius: all near values against the dense fill, a sample against the
    oracle."""
    import torch

    V, F = meshes.icosphere(5)
    k, Q = 17.0, 7
    r = 0.25 * 2 * np.pi / k
    m = mf.Mesh(F, V.shape[0])
    nf = mf.NearField(m, V, r)
    say("near ico5", nf.nnz, "pairs", nf.n_tiles, "tiles")
    lo, hi = mf.r_range(m, V, Q)
    T = mf.build_tables(k, lo, hi, 1e-5)
    vals = nf.fill(V, k, Q, "table", T)
    Z = mf.fill_Z(m, V, k, Q, "table", T)
    mf.sync_status(m)
    rows, cols = _coo(*nf.pattern())
    rt, ct = torch.tensor(rows, device="cuda"), torch.tensor(cols, device="cuda")
    e_dense = float((vals - Z[rt, ct]).abs().norm() / Z[rt, ct].abs().norm())
    del Z
    rng = np.random.default_rng(77)
    pick = rng.choice(nf.nnz, 3000, replace=False)
    ref = orc.fill_entries(V, F, m.edges(), k, Q, rows[pick], cols[pick])
    e_orc = _rel(vals.cpu().numpy()[pick], ref)
    say(f"  vs dense {e_dense:.2e}, sampled vs oracle {e_orc:.2e}")
    assert e_dense <= 1e-6
    assert e_orc <= 1e-5
