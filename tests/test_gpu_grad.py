"""GPU parity of the adjoint: dL/dV and dL/dk of L = Re sum conj(W) Z from
the HIP backward against the oracle's finite-difference gradient of its FP64
loss, plus the invariants the matrix forces at full size (translation,
rotation, the homogeneity Z(aV, k/a) = a^2 Z(V, k)), and the autograd path.

Tolerances.  The regular pairs are summed in FP32 (unit roundoff 6e-8):
with the FP64 centroid offset split in two floats, each term of a vertex's
sum carries a relative error of a few units of roundoff and the sum over
its pairs cancels by about one decade, so the gradient is held to 3e-6 of
its largest component (50 units).  Table mode differentiates the
interpolating cubic, whose derivative error is of order tol/t (t the
sample spacing) rather than tol; with tol = 1e-8 and t near 1e-2 that is
1e-6, inside the same bound.  The invariants are sums over every vertex
and hold to 1e-7 of the sum of magnitudes."""

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


def _small():
    V, F = meshes.icosphere(1)
    V = meshes.jitter_uniform(V, F, 0.08, 11)
    return V, F, 3.0, 6


@pytest.fixture(scope="module")
def small_ref(orc):
    V, F, k, Q = _small()
    edges = orc.rwg(V, F)
    W = meshes.dual_weights(edges.shape[0], 21)
    g, gk = orc.grad_fd(V, F, edges, k, Q, W)
    return V, F, k, Q, W, g.reshape(-1, 3), gk


@pytest.mark.parametrize("wdtype", ["c128", "c64"])
def test_grad_direct_small(mf, small_ref, wdtype):
    import torch

    V, F, k, Q, W, g_ref, gk_ref = small_ref
    say("grad direct small", wdtype)
    m = mf.Mesh(F, V.shape[0])
    dt = torch.complex128 if wdtype == "c128" else torch.complex64
    Wd = torch.tensor(W, dtype=dt, device="cuda")
    if wdtype == "c64":  # the oracle sees the same rounded weights
        W = Wd.cpu().numpy().astype(np.complex128)
        from oracle import grad_fd, rwg

        g, gk_ref = grad_fd(V, F, rwg(V, F), k, Q, W)
        g_ref = g.reshape(-1, 3)
    dV, dk = mf.fill_Z_backward(m, V, k, Q, "direct", None, Wd)
    dV = dV.cpu().numpy()
    err = np.abs(dV - g_ref).max() / np.abs(g_ref).max()
    errk = abs(float(dk.item()) - gk_ref) / abs(gk_ref)
    say(f"  vertex err {err:.3e}, dk err {errk:.3e}")
    assert err <= 3e-6
    assert errk <= 3e-6


def test_grad_table_small(mf, small_ref):
    import torch

    V, F, k, Q, W, g_ref, gk_ref = small_ref
    say("grad table small")
    m = mf.Mesh(F, V.shape[0])
    lo, hi = mf.r_range(m, V, Q)
    T = mf.build_tables(k, lo, hi, 1e-8)
    Wd = torch.tensor(W, dtype=torch.complex128, device="cuda")
    dV, dk = mf.fill_Z_backward(m, V, k, Q, "table", T, Wd)
    dV = dV.cpu().numpy()
    err = np.abs(dV - g_ref).max() / np.abs(g_ref).max()
    errk = abs(float(dk.item()) - gk_ref) / abs(gk_ref)
    say(f"  vertex err {err:.3e}, dk err {errk:.3e}")
    assert err <= 3e-6
    assert errk <= 3e-6


def test_grad_only_touching_pairs(mf, orc):
    """A tetrahedron has no regular pairs: the whole gradient comes from the
    FP64 touching-pair kernel."""
    import torch

    V = np.array([[0.0, 0.0, 0.0], [0.3, 0.0, 0.02], [0.05, 0.28, 0.0], [0.1, 0.08, 0.25]])
    F = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [2, 0, 3]], dtype=np.int32)
    k, Q = 5.0, 7
    say("grad tetrahedron")
    edges = orc.rwg(V, F)
    W = meshes.dual_weights(edges.shape[0], 3)
    g_ref, gk_ref = orc.grad_fd(V, F, edges, k, Q, W)
    m = mf.Mesh(F, V.shape[0])
    dV, dk = mf.fill_Z_backward(m, V, k, Q, "direct", None,
                                torch.tensor(W, dtype=torch.complex128, device="cuda"))
    err = np.abs(dV.cpu().numpy().ravel() - g_ref).max() / np.abs(g_ref).max()
    say(f"  vertex err {err:.3e}")
    assert err <= 1e-8
    assert abs(float(dk.item()) - gk_ref) <= 1e-8 * abs(gk_ref)


@pytest.fixture(scope="module")
def ico4(mf):
    import torch

    wl = meshes.workload("ico4_grad")
    V, F, k, Q = wl["V"], wl["F"], wl["k"], wl["Q"]
    m = mf.Mesh(F, V.shape[0])
    E = m.n_edges
    W = torch.complex(torch.randn(E, E, dtype=torch.float32, generator=torch.Generator().manual_seed(8)),
                      torch.randn(E, E, dtype=torch.float32,
                                  generator=torch.Generator().manual_seed(9))).cuda()
    return V, F, k, Q, m, W


@pytest.mark.parametrize("mode", ["direct", "table"])
def test_grad_invariants_full_size(mf, ico4, mode):
    """Translation and rotation invariance and the scaling identity
    sum x.dL/dx - k dL/dk = 2L on the 7,680-unknown jittered sphere."""
    import torch

    V, F, k, Q, m, W = ico4
    say("grad invariants ico4", mode)
    T = None
    if mode == "table":
        lo, hi = mf.r_range(m, V, Q)
        T = mf.build_tables(k, lo, hi, 1e-8)
    Z = mf.fill_Z(m, V, k, Q, mode, T, dtype=torch.complex64)
    L = float(torch.real(torch.conj(W) * Z).double().sum().item())
    dV, dk = mf.fill_Z_backward(m, V, k, Q, mode, T, W)
    g = dV.cpu().numpy()
    gk = float(dk.item())
    scale = np.abs(g).sum()
    t = np.abs(g.sum(0)).max() / scale
    r = np.abs(np.cross(V, g).sum(0)).max() / scale
    lhs = float((V * g).sum()) - k * gk
    e = abs(lhs - 2 * L) / (np.abs(V * g).sum() + abs(k * gk) + abs(L))
    say(f"  translation {t:.2e} rotation {r:.2e} scaling {e:.2e}")
    assert t <= 1e-7 and r <= 1e-7
    # table mode holds the tables fixed: the identity holds to the table tolerance
    assert e <= 1e-7


def test_grad_sampled_full_size(mf, orc, ico4):
    """Sampled vertex coordinates of the 7,680-unknown case against the
    oracle's finite differences of its local loss."""
    V, F, k, Q, m, W = ico4
    say("grad sampled ico4")
    dV, _ = mf.fill_Z_backward(m, V, k, Q, "direct", None, W)
    g = dV.cpu().numpy().ravel()
    Wn = W.cpu().numpy().astype(np.complex128)
    rng = np.random.default_rng(12)
    idx = rng.choice(V.size, 4, replace=False)
    ref, _ = orc.grad_fd(V, F, m.edges(), k, Q, Wn, idx, with_k=False)
    err = np.abs(g[idx] - ref).max() / np.abs(g).max()
    say(f"  sampled err {err:.3e}")
    assert err <= 3e-6


def test_autograd_path(mf):
    import torch

    V, F, k, Q = _small()
    say("autograd")
    m = mf.Mesh(F, V.shape[0])
    E = m.n_edges
    W = torch.tensor(meshes.dual_weights(E, 30), dtype=torch.complex128, device="cuda")
    Vt = torch.tensor(V, dtype=torch.float64, device="cuda", requires_grad=True)
    kt = torch.tensor(k, dtype=torch.float64, requires_grad=True)
    Z = mf.fill(Vt, kt, m, Q, "direct", dtype=torch.complex128)
    L = torch.real(torch.conj(W) * Z).sum()
    L.backward()
    dV, dk = mf.fill_Z_backward(m, V, k, Q, "direct", None, W)
    # same kernels; FP64 atomics may add in another order
    assert torch.allclose(Vt.grad, dV, rtol=1e-10, atol=1e-12 * float(dV.abs().max()))
    assert abs(float(kt.grad) - float(dk.item())) <= 1e-10 * abs(float(dk.item()))


@pytest.fixture(scope="module")
def ico4_fd(orc, ico4):
    """Finite-difference reference of the 7,680-unknown case on the FP64
    oracle (direct exponential): dL/dV at 64 seeded coordinates (local loss,
    central differences with one Richardson step), dL/dk (full loss filled in
    triangle-pair order, Richardson), and the derivatives along 8 seeded
    random unit directions in the 7,686-dimensional space of the coordinates
    (full loss, central differences, h = 1e-4)."""
    V, F, k, Q, m, W = ico4
    E = m.edges()
    Wn = W.cpu().numpy().astype(np.complex128)
    rng = np.random.default_rng(12)
    idx = np.sort(rng.choice(V.size, 64, replace=False))
    say("oracle FD: 64 coordinates")
    g_idx, _ = orc.grad_fd(V, F, E, k, Q, Wn, idx, with_k=False)

    def loss(Vx, kx):
        Z = orc.fill_rows(Vx, F, E, kx, Q, 0, E.shape[0])
        return float(np.sum(np.real(np.conj(Wn) * Z)))

    say("oracle FD: dL/dk")
    hk = 1e-4 * k
    d = [(loss(V, k + hh) - loss(V, k - hh)) / (2 * hh) for hh in (hk, hk / 2)]
    gk = (4 * d[1] - d[0]) / 3
    D = np.random.default_rng(13).standard_normal((8, V.size))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    h = 1e-4
    dd = np.zeros(8)
    for i in range(8):
        say("oracle FD: direction", i)
        step = D[i].reshape(V.shape)
        dd[i] = (loss(V + h * step, k) - loss(V - h * step, k)) / (2 * h)
    return idx, g_idx, gk, D, dd


@pytest.mark.parametrize("mode,tol,bar", [("direct", None, 1e-5), ("table", 1e-6, 1e-4)])
def test_grad_against_fd_full_size(mf, ico4, ico4_fd, mode, tol, bar):
    """The adjoint of the 7,680-unknown jittered sphere (k = 10, 6-point rule,
    W complex64 N(0,1)) against the oracle's finite differences: 64 vertex
    coordinates, 8 random directions and dL/dk, each error relative to the
    norm of its reference.  Table mode holds its tables fixed and
    differentiates the interpolant, so its bar carries the table's own
    derivative error."""
    V, F, k, Q, m, W = ico4
    idx, g_idx, gk_ref, D, dd = ico4_fd
    T = None
    if mode == "table":
        lo, hi = mf.r_range(m, V, Q)
        T = mf.build_tables(k, lo, hi, tol)
    say("adjoint", mode)
    dV, dk = mf.fill_Z_backward(m, V, k, Q, mode, T, W)
    g = dV.cpu().numpy().ravel()
    e_coord = np.linalg.norm(g[idx] - g_idx) / np.linalg.norm(g_idx)
    e_dir = np.linalg.norm(D @ g - dd) / np.linalg.norm(dd)
    e_k = abs(float(dk.item()) - gk_ref) / abs(gk_ref)
    say(f"  {mode}: 64 coordinates {e_coord:.3e}, 8 directions {e_dir:.3e}, dL/dk {e_k:.3e}")
    assert e_coord <= bar and e_dir <= bar and e_k <= bar
