"""Run-to-run determinism of the EFIE fills.

The regular-pair accumulation is atomic-free in every EFIE fill kernel (the
triangle-block tiles, the cut-edge fix-up, the edge-block tiles and the
batched launch), so two fills of the same inputs must agree bit for bit.
The output is poisoned with NaN before each fill so that an entry the fill
leaves unwritten cannot pass as equal.  (The MFIE's non-owner halves, the
angular inner integrals and the adjoint's FP64 sums use atomics and are
reproducible only to rounding; they are not checked here.)
"""

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


def _bits(Z):
    import torch

    return torch.view_as_real(Z).contiguous().view(torch.int32 if Z.dtype == torch.complex64
                                                   else torch.int64)


def _twice(fn, E, dtype):
    import torch

    out = []
    for _ in range(2):
        Z = torch.full((E, E), float("nan"), dtype=dtype, device="cuda")
        fn(Z)
        torch.cuda.synchronize()
        assert not torch.isnan(torch.view_as_real(Z)).any()
        out.append(_bits(Z))
    return out


@pytest.mark.parametrize("mode", ["table", "direct"])
def test_fill_bitwise_reproducible(mf, mode):
    import torch

    V, F = meshes.icosphere(4)
    k, Q, tol = 10.0, 6, 1e-6
    m = mf.Mesh(F, V.shape[0])
    E = m.n_edges
    lo, hi = mf.r_range(m, V, Q)
    T = mf.build_tables(k, lo, hi, tol) if mode == "table" else None
    say("ico4", mode, "E", E)
    a, b = _twice(lambda Z: mf.fill_Z(m, V, k, Q, mode, T, out=Z), E, torch.complex64)
    assert torch.equal(a, b)
    if mode == "table":
        # every kernel the tuner can choose, pinned in turn
        for c in range(3):
            name = mf.lib().mf_fill_choice_name(c).decode()
            say("choice", c, name)
            m.set_fill_choice(c)
            x, y = _twice(lambda Z: mf.fill_Z(m, V, k, Q, mode, T, out=Z), E, torch.complex64)
            assert torch.equal(x, y), name
        m.set_fill_choice(-1)


def test_batch_bitwise_reproducible(mf):
    import torch

    k, Q, tol = 6.0, 6, 1e-6
    items = []
    for s, seed in ((3, 1), (3, 2)):
        V, F = meshes.icosphere(s)
        V = meshes.jitter_uniform(V, F, 0.05, seed)
        m = mf.Mesh(F, V.shape[0])
        lo, hi = mf.r_range(m, V, Q)
        items.append((m, V, mf.build_tables(k, lo, hi, tol)))
    runs = []
    for _ in range(2):
        Zs = [torch.full((m.n_edges, m.n_edges), float("nan"), dtype=torch.complex64,
                         device="cuda") for m, _, _ in items]
        mf.Batch([(m, V, k, T, Z) for (m, V, T), Z in zip(items, Zs)], Q, "table").fill()
        torch.cuda.synchronize()
        runs.append([_bits(Z) for Z in Zs])
    for x, y in zip(*runs):
        assert torch.equal(x, y)
