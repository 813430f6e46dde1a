"""The allocation-free range scan (scratch in the library's static device
array) against the workspace entry point, through the C-ABI: two calls in a
row on one GPU, the second on a smaller mesh, bit for bit."""

import ctypes as C
import sys

import numpy as np
import pytest

from paper_1901_04162_amd import meshes

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_static_scratch_range_matches_workspace_range():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1901_04162_amd as mf

    L = mf.lib()
    s = mf._stream()
    for name, (V, F), q in (("ico4", meshes.icosphere(4), 7), ("ico2", meshes.icosphere(2), 3)):
        say("range", name, "triangles", F.shape[0])
        m = mf.Mesh(F, V.shape[0])
        Vd = torch.tensor(V, dtype=torch.float64, device="cuda")
        lo, hi = C.c_double(), C.c_double()
        slo, shi = C.c_double(), C.c_double()
        mf.check(L.mf_r_range(m.device_handle, C.c_void_p(Vd.data_ptr()), q, C.byref(lo),
                              C.byref(hi), s))
        mf.check(L.mf_r_range_static(m.device_handle, C.c_void_p(Vd.data_ptr()), q,
                                     C.byref(slo), C.byref(shi), s))
        say(name, lo.value, hi.value, slo.value, shi.value)
        assert (slo.value, shi.value) == (lo.value, hi.value)
        assert np.isfinite(lo.value) and 0.0 < lo.value < hi.value
