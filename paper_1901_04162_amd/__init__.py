"""MI355X EFIE impedance-matrix fill with adaptive Green-function tables.

Python face of libmomfill.so: torch supplies device memory and the stream,
every step of the fill runs in the library's HIP kernels.
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as _L
from ._lib import (MF_C64, MF_C128, MF_MODE_DIRECT, MF_MODE_TABLE, MF_PART_A,  # noqa: F401
                   MF_PART_PHI, MomfillError, check, lib)

MODES = {"table": MF_MODE_TABLE, "direct": MF_MODE_DIRECT}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Mesh:
    """Topology of a triangle mesh (RWG edges, touching pairs, tile plan)."""

    def __init__(self, F, n_vertices: int):
        F = np.ascontiguousarray(np.asarray(F), dtype=np.int32)
        if F.ndim != 2 or F.shape[1] != 3:
            raise ValueError("F must be (n_triangles, 3)")
        h = C.c_void_p()
        check(lib().mf_mesh_create(int(n_vertices), F.shape[0],
                                   F.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(h)))
        self._h = h
        self.n_vertices = int(n_vertices)
        self.n_triangles = F.shape[0]
        n = C.c_int32()
        check(lib().mf_mesh_n_edges(h, C.byref(n)))
        self.n_edges = n.value

    @property
    def handle(self):
        return self._h

    @property
    def device_handle(self):
        """The handle with its device workspace bound: a torch tensor of the
        size the library asks for, made on first use (the library allocates
        no device memory itself)."""
        if getattr(self, "_ws", None) is None:
            n = C.c_size_t()
            check(lib().mf_mesh_workspace_bytes(self._h, C.byref(n)))
            ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device="cuda")
            check(lib().mf_mesh_set_workspace(self._h, C.c_void_p(ws.data_ptr()), n.value,
                                              _stream()))
            self._ws = ws
        return self._h

    def edges(self) -> np.ndarray:
        out = np.zeros((self.n_edges, 6), dtype=np.int32)
        check(lib().mf_mesh_edges(self._h, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def n_touching(self) -> int:
        n = C.c_int64()
        check(lib().mf_mesh_n_touching(self._h, C.byref(n)))
        return n.value

    def tb_plan(self):
        """(blocks, tiles, cut edges, largest number of rounds) of the
        triangle-block plan of the table-mode fill (zeros: no such plan)."""
        nb, nc, mr = C.c_int32(), C.c_int32(), C.c_int32()
        nt = C.c_int64()
        check(lib().mf_mesh_tb_plan(self._h, C.byref(nb), C.byref(nt), C.byref(nc), C.byref(mr)))
        return nb.value, nt.value, nc.value, mr.value

    def set_fill_choice(self, choice: int):
        """Pins the kernel of table-mode fills (0, 1, 2: see
        mf_fill_choice_name; -1: cached choice or kernel 0)."""
        check(lib().mf_mesh_set_fill_choice(self._h, int(choice)))

    def plan(self):
        """(blocks, tiles, largest triangles per block) of the regular fill."""
        nb, mt = C.c_int32(), C.c_int32()
        nt = C.c_int64()
        check(lib().mf_mesh_plan(self._h, C.byref(nb), C.byref(nt), C.byref(mt)))
        return nb.value, nt.value, mt.value

    def __del__(self, _L=_L):
        if getattr(self, "_h", None) and _L._lib is not None:
            _L._lib.mf_mesh_destroy(self._h)
            self._h = None


class Tables:
    """Device tables of Exp(-jkr) (linear) and Exp(-jkr)/r (cubic Lagrange)."""

    def __init__(self, k: float, r_min: float, r_max: float, tol: float, exp_only: bool = False):
        h = C.c_void_p()
        n = C.c_size_t()
        if exp_only:
            if r_min != 0.0:
                raise ValueError("the Exp table alone starts at r = 0")
            check(lib().mf_exp_table_workspace_bytes(float(k), float(r_max), float(tol),
                                                     C.byref(n)))
        else:
            check(lib().mf_tables_workspace_bytes(float(k), float(r_min), float(r_max),
                                                  float(tol), C.byref(n)))
        # the tables live in this tensor (the library allocates no device memory)
        self._ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device="cuda")
        wsp = C.c_void_p(self._ws.data_ptr())
        if exp_only:
            check(lib().mf_build_exp_table(float(k), float(r_max), float(tol), wsp, n.value,
                                           C.byref(h), _stream()))
        else:
            check(lib().mf_build_tables(float(k), float(r_min), float(r_max), float(tol), wsp,
                                        n.value, C.byref(h), _stream()))
        self._h = h
        self.k, self.r_min, self.r_max, self.tol = float(k), float(r_min), float(r_max), float(tol)
        ne, ng, me, mg = (C.c_int32() for _ in range(4))
        te, tg, ee, eg = (C.c_double() for _ in range(4))
        check(lib().mf_tables_info(h, C.byref(ne), C.byref(ng), C.byref(me), C.byref(mg),
                                   C.byref(te), C.byref(tg), C.byref(ee), C.byref(eg)))
        self.n_exp, self.n_green, self.m_exp, self.m_green = ne.value, ng.value, me.value, mg.value
        self.t_exp, self.t_green, self.err_exp, self.err_green = te.value, tg.value, ee.value, eg.value

    @property
    def handle(self):
        return self._h

    def get(self, which: str):
        """(nodes, values, hash) of the 'exp' or 'green' table as numpy arrays."""
        w = 0 if which == "exp" else 1
        n = self.n_exp if w == 0 else self.n_green
        m = self.m_exp if w == 0 else self.m_green
        r = np.zeros(n)
        f = np.zeros(2 * n)
        h = np.zeros(m, dtype=np.int32)
        dp = C.POINTER(C.c_double)
        check(lib().mf_tables_get(self._h, w, r.ctypes.data_as(dp), f.ctypes.data_as(dp),
                                  h.ctypes.data_as(C.POINTER(C.c_int32)), _stream()))
        return r, f[0::2] + 1j * f[1::2], h

    def eval(self, which: str, r: torch.Tensor) -> torch.Tensor:
        """FP32 lookup + interpolation at device points r (float64)."""
        r = r.to(device="cuda", dtype=torch.float64).contiguous()
        out = torch.empty(r.numel(), dtype=torch.complex128, device="cuda")
        check(lib().mf_tables_eval(self._h, 0 if which == "exp" else 1, r.numel(),
                                   C.c_void_p(r.data_ptr()), C.c_void_p(out.data_ptr()),
                                   _stream()))
        return out

    def __del__(self, _L=_L):
        if getattr(self, "_h", None) and _L._lib is not None:
            _L._lib.mf_tables_destroy(self._h)
            self._h = None


def _vertices(V) -> torch.Tensor:
    if not isinstance(V, torch.Tensor):
        V = torch.as_tensor(np.asarray(V, dtype=np.float64))
    return V.to(device="cuda", dtype=torch.float64).contiguous()


def r_range(mesh: Mesh, V, quad_order: int):
    """Exact FP64 (r_min, r_max) over regular quadrature-point pairs."""
    Vd = _vertices(V)
    lo, hi = C.c_double(), C.c_double()
    check(lib().mf_r_range(mesh.device_handle, C.c_void_p(Vd.data_ptr()), int(quad_order),
                           C.byref(lo), C.byref(hi), _stream()))
    return lo.value, hi.value


def build_tables(k: float, r_min: float, r_max: float, tol: float) -> Tables:
    return Tables(k, r_min, r_max, tol)


def angular_rmax(mesh: Mesh, V, quad_order: int) -> float:
    """Largest quadrature-point-to-vertex distance (exact, FP64): the upper
    end of the Exp table of the angular-transformation fill."""
    Vd = _vertices(V)
    out = C.c_double()
    check(lib().mf_angular_rmax(mesh.device_handle, C.c_void_p(Vd.data_ptr()), int(quad_order),
                                C.byref(out), _stream()))
    return out.value


def build_exp_table(k: float, r_max: float, tol: float) -> Tables:
    """The linear Exp(-jkr) table alone, over [0, r_max]."""
    return Tables(k, 0.0, r_max, tol, exp_only=True)


def fill_angular(mesh: Mesh, V, k: float, quad_order: int, n_edge: int = 8,
                 mode: str = "table", table: Tables = None, dtype=torch.complex64,
                 out: torch.Tensor = None) -> torch.Tensor:
    """EFIE matrix with every inner integral by the angular transformation
    (n_edge points per source edge, FP64 integrals)."""
    Vd = _vertices(V)
    out, zt = _z_out(mesh, dtype, out)
    check(lib().mf_fill_angular(mesh.device_handle, C.c_void_p(Vd.data_ptr()), float(k),
                                int(quad_order), int(n_edge), MODES[mode],
                                table.handle if table is not None else None,
                                C.c_void_p(out.data_ptr()), zt, out.stride(0), _stream()))
    return out


def _z_out(mesh: Mesh, dtype, out):
    E = mesh.n_edges
    if out is None:
        out = torch.empty((E, E), dtype=dtype, device="cuda")
    if out.dtype not in (torch.complex64, torch.complex128) or out.dim() != 2 or \
            out.shape[0] < E or out.shape[1] < E or out.stride(1) != 1:
        raise ValueError("out must be a row-major complex64/complex128 matrix of at least E x E")
    return out, (MF_C64 if out.dtype == torch.complex64 else MF_C128)


def fill_Z(mesh: Mesh, V, k: float, quad_order: int, mode: str = "table", tables: Tables = None,
           dtype=torch.complex64, out: torch.Tensor = None, part: int = 0) -> torch.Tensor:
    """Impedance matrix Z (n_edges x n_edges) on the current device."""
    Vd = _vertices(V)
    out, zt = _z_out(mesh, dtype, out)
    m = MODES[mode] | part
    check(lib().mf_fill_Z(mesh.device_handle, C.c_void_p(Vd.data_ptr()), float(k), int(quad_order), m,
                          tables.handle if tables is not None else None,
                          C.c_void_p(out.data_ptr()), zt, out.stride(0), _stream()))
    return out


def tune_fill(mesh: Mesh, V, k: float, quad_order: int, mode: str = "table",
              tables: Tables = None, dtype=torch.complex64, out: torch.Tensor = None):
    """Times the kernels a fill of these arguments can run on, keeps the
    fastest for this mesh (and in the MOMFILL_TUNE_CACHE file when set).
    Returns (Z, choice, description, [ms per kernel]); Z holds the fill."""
    Vd = _vertices(V)
    Z, zt = _z_out(mesh, dtype, out)
    ch = C.c_int32()
    ms = (C.c_float * 3)()
    check(lib().mf_fill_tune(mesh.device_handle, C.c_void_p(Vd.data_ptr()), float(k),
                             int(quad_order), MODES[mode],
                             tables.handle if tables is not None else None,
                             C.c_void_p(Z.data_ptr()), zt, Z.stride(0), _stream(), C.byref(ch),
                             ms))
    return Z, ch.value, lib().mf_fill_choice_name(ch.value).decode(), [float(x) for x in ms]


def fill_mfie(mesh: Mesh, V, k: float, quad_order: int, mode: str = "table",
              tables: Tables = None, dtype=torch.complex64,
              out: torch.Tensor = None) -> torch.Tensor:
    """MFIE matrix <f_m, f_n>/2 - K_mn (n_edges x n_edges) on the current device."""
    Vd = _vertices(V)
    out, zt = _z_out(mesh, dtype, out)
    check(lib().mf_fill_mfie(mesh.device_handle, C.c_void_p(Vd.data_ptr()), float(k), int(quad_order),
                             MODES[mode], tables.handle if tables is not None else None,
                             C.c_void_p(out.data_ptr()), zt, out.stride(0), _stream()))
    return out


def _rhs(fn, mesh: Mesh, V, k, quad_order, khat, E0, dtype):
    Vd = _vertices(V)
    kh = np.ascontiguousarray(np.asarray(khat, dtype=np.float64))
    e0 = np.asarray(E0, dtype=np.complex128)
    e0 = np.ascontiguousarray(np.stack([e0.real, e0.imag], 1).ravel())
    out = torch.empty(mesh.n_edges, dtype=dtype, device="cuda")
    dp = C.POINTER(C.c_double)
    check(fn(mesh.device_handle, C.c_void_p(Vd.data_ptr()), float(k), int(quad_order),
             kh.ctypes.data_as(dp), e0.ctypes.data_as(dp), C.c_void_p(out.data_ptr()),
             MF_C64 if dtype == torch.complex64 else MF_C128, _stream()))
    return out


def rhs_planewave(mesh: Mesh, V, k: float, quad_order: int, khat, E0,
                  dtype=torch.complex64) -> torch.Tensor:
    """V_m = int f_m . E0 exp(-j k khat.r) dS on the current device."""
    return _rhs(lib().mf_rhs_planewave, mesh, V, k, quad_order, khat, E0, dtype)


def rhs_planewave_mfie(mesh: Mesh, V, k: float, quad_order: int, khat, E0,
                       dtype=torch.complex64) -> torch.Tensor:
    """V_m = int f_m . (n x H_inc) dS, H_inc = khat x E0 exp(-j k khat.r)/eta0."""
    return _rhs(lib().mf_rhs_planewave_mfie, mesh, V, k, quad_order, khat, E0, dtype)


def far_field(mesh: Mesh, V, k: float, quad_order: int, I: torch.Tensor, dirs, e0_norm=1.0):
    """(F [n,3] complex128, sigma [n] float64) for currents I in unit directions dirs."""
    Vd = _vertices(V)
    d = torch.as_tensor(np.asarray(dirs, dtype=np.float64)).to("cuda").contiguous()
    I = I.contiguous()
    n = d.shape[0]
    F = torch.empty((n, 3), dtype=torch.complex128, device="cuda")
    sig = torch.empty(n, dtype=torch.float64, device="cuda")
    check(lib().mf_far_field(mesh.device_handle, C.c_void_p(Vd.data_ptr()), float(k), int(quad_order),
                             C.c_void_p(I.data_ptr()),
                             MF_C64 if I.dtype == torch.complex64 else MF_C128, n,
                             C.c_void_p(d.data_ptr()), float(e0_norm),
                             C.c_void_p(F.data_ptr()), C.c_void_p(sig.data_ptr()), _stream()))
    return F, sig


class NearField:
    """CSR pattern of the near-field unknown pairs (edge midpoints at most
    r_near apart) and the fill of their entries."""

    def __init__(self, mesh: Mesh, V, r_near: float):
        Vh = np.ascontiguousarray(np.asarray(V, dtype=np.float64))
        self._h = C.c_void_p()
        check(lib().mf_near_create(mesh.handle, Vh.ctypes.data_as(C.POINTER(C.c_double)),
                                   float(r_near), C.byref(self._h)))
        self.mesh = mesh
        nnz, nt = C.c_int64(), C.c_int64()
        check(lib().mf_near_info(self._h, C.byref(nnz), C.byref(nt)))
        self.nnz, self.n_tiles = nnz.value, nt.value

    def pattern(self):
        """(row_ptr int64 [E+1], col int32 [nnz]) on the host."""
        rp = np.zeros(self.mesh.n_edges + 1, dtype=np.int64)
        col = np.zeros(max(self.nnz, 1), dtype=np.int32)
        check(lib().mf_near_pattern(self._h, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                    col.ctypes.data_as(C.POINTER(C.c_int32))))
        return rp, col[:self.nnz]

    def fill(self, V, k: float, quad_order: int, mode: str = "table", tables: Tables = None,
             dtype=torch.complex64, out: torch.Tensor = None) -> torch.Tensor:
        Vd = _vertices(V)
        if out is None:
            out = torch.empty(self.nnz, dtype=dtype, device="cuda")
        if out.dtype not in (torch.complex64, torch.complex128) or out.numel() < self.nnz or \
                not out.is_contiguous():
            raise ValueError("out must be a contiguous complex vector of nnz values")
        zt = MF_C64 if out.dtype == torch.complex64 else MF_C128
        if getattr(self, "_ws", None) is None:
            n = C.c_size_t()
            check(lib().mf_near_workspace_bytes(self._h, C.byref(n)))
            self._ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device="cuda")
            check(lib().mf_near_set_workspace(self._h, C.c_void_p(self._ws.data_ptr()), n.value,
                                              _stream()))
        check(lib().mf_fill_near(self.mesh.device_handle, self._h, C.c_void_p(Vd.data_ptr()), float(k),
                                 int(quad_order), MODES[mode],
                                 tables.handle if tables is not None else None,
                                 C.c_void_p(out.data_ptr()), zt, _stream()))
        return out

    def __del__(self, _L=_L):
        if getattr(self, "_h", None) and _L._lib is not None:
            _L._lib.mf_near_destroy(self._h)
            self._h = None


class Batch:
    """One persistent fill launch over several (mesh, k) items.

    items: sequence of (mesh, V, k, tables, Z), Z a row-major complex tensor
    of at least E x E on the current device.  All items share quad_order,
    mode and the dtype of Z; items sharing a mesh must share V (the same
    device tensor).  The tensors must stay alive while the batch exists.
    fill() only enqueues kernels (no allocation, no copy), so it can be
    captured in a CUDA graph.
    """

    def __init__(self, items, quad_order: int, mode: str = "table"):
        items = list(items)
        n = len(items)
        if n < 1:
            raise ValueError("empty batch")
        self._keep = []
        zt = None
        meshes, vps, ks, tps, zps, lds = [], [], [], [], [], []
        for mesh, V, k, tables, Z in items:
            Vd = _vertices(V)  # the library checks that a shared mesh has one V
            if Z.dtype not in (torch.complex64, torch.complex128) or Z.dim() != 2 or \
                    Z.stride(1) != 1 or Z.shape[0] < mesh.n_edges or Z.shape[1] < mesh.n_edges:
                raise ValueError("each Z must be a row-major complex matrix of at least E x E")
            t = MF_C64 if Z.dtype == torch.complex64 else MF_C128
            if zt is not None and t != zt:
                raise ValueError("all outputs of a batch share one dtype")
            zt = t
            meshes.append(mesh.device_handle.value)
            vps.append(Vd.data_ptr())
            ks.append(float(k))
            tps.append(tables.handle.value if tables is not None else None)
            zps.append(Z.data_ptr())
            lds.append(Z.stride(0))
            self._keep += [mesh, Vd, tables, Z]
        arr = C.c_void_p * n
        self._h = C.c_void_p()
        nb = C.c_size_t()
        check(lib().mf_batch_workspace_bytes(n, arr(*meshes), C.byref(nb)))
        self._ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device="cuda")
        check(lib().mf_batch_create(n, arr(*meshes), arr(*vps), (C.c_double * n)(*ks),
                                    arr(*tps) if mode == "table" else None, int(quad_order),
                                    MODES[mode], arr(*zps), zt, (C.c_int64 * n)(*lds),
                                    C.c_void_p(self._ws.data_ptr()), nb.value,
                                    C.byref(self._h)))
        self.n = n

    def fill(self):
        check(lib().mf_batch_fill(self._h, _stream()))

    # the tuner's candidates, in the order of its timings
    CANDIDATES = (("edge", 512), ("edge", 768), ("edge", 1024), ("triangle", 1024),
                  ("triangle", 512))

    def tuning(self):
        """(tile shape picked by the tuner, "edge" or "triangle" blocks,
        threads per workgroup, its timings in ms for CANDIDATES; zeros for
        candidates not run and when an earlier batch's choice was reused)."""
        t = C.c_int32()
        sh = C.c_int32()
        ms = (C.c_float * len(self.CANDIDATES))()
        check(lib().mf_batch_info(self._h, C.byref(t), C.byref(sh), ms))
        return ("edge", "triangle")[sh.value], t.value, [float(v) for v in ms]

    def set_choice(self, shape: str, threads: int):
        """Pins the launch to one of CANDIDATES for later fill() calls."""
        check(lib().mf_batch_set_choice(self._h, self.CANDIDATES.index((shape, int(threads)))))

    def __del__(self, _L=_L):
        if getattr(self, "_h", None) and _L._lib is not None:
            _L._lib.mf_batch_destroy(self._h)
            self._h = None


def set_timing(on: bool):
    lib().mf_set_timing(1 if on else 0)


def timings(mesh: Mesh):
    """(geometry, touching pairs, regular fill) milliseconds of the last timed fill."""
    ms = (C.c_float * 3)()
    check(lib().mf_mesh_timings(mesh.device_handle, ms))
    return tuple(float(x) for x in ms)


def fill_timings(mesh: Mesh):
    """(tile kernel, cut-edge fix-up) milliseconds of the last timed fill's
    regular phase (fix-up 0 when the fill had none)."""
    ms = (C.c_float * 2)()
    check(lib().mf_mesh_fill_timings(mesh.device_handle, ms))
    return float(ms[0]), float(ms[1])


def sync_status(mesh: Mesh):
    check(lib().mf_sync_status(mesh.device_handle, _stream()))


def fill_Z_backward(mesh: Mesh, V, k: float, quad_order: int, mode: str, tables: Tables,
                    dLdZ: torch.Tensor):
    """(dL/dV [nv,3] float64, dL/dk float) for L = Re sum conj(dLdZ) * Z."""
    Vd = _vertices(V)
    W = dLdZ.contiguous()
    zt = MF_C64 if W.dtype == torch.complex64 else MF_C128
    dV = torch.empty_like(Vd)
    dk = torch.empty(1, dtype=torch.float64, device="cuda")
    check(lib().mf_fill_Z_backward(mesh.device_handle, C.c_void_p(Vd.data_ptr()), float(k),
                                   int(quad_order), MODES[mode],
                                   tables.handle if tables is not None else None,
                                   C.c_void_p(W.data_ptr()), zt, W.stride(0),
                                   C.c_void_p(dV.data_ptr()), C.c_void_p(dk.data_ptr()),
                                   _stream()))
    return dV, dk


class _FillFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, k, mesh, quad_order, mode, tables, dtype):
        Z = fill_Z(mesh, V, float(k), quad_order, mode, tables, dtype)
        ctx.save_for_backward(V)
        ctx.meta = (float(k), mesh, quad_order, mode, tables)
        ctx.k_like = (k.device, k.dtype) if isinstance(k, torch.Tensor) else (None, None)
        return Z

    @staticmethod
    def backward(ctx, gZ):
        (V,) = ctx.saved_tensors
        k, mesh, quad_order, mode, tables = ctx.meta
        # torch hands the gradient of a real loss w.r.t. complex Z as dL/dRe + j dL/dIm,
        # which is the W of L = Re sum conj(W) Z
        dV, dk = fill_Z_backward(mesh, V, k, quad_order, mode, tables, gZ)
        kdev, kdt = ctx.k_like
        dk = dk.reshape(()) if kdev is None else dk.reshape(()).to(device=kdev, dtype=kdt)
        return dV.to(V.dtype), dk, None, None, None, None, None


def fill(V: torch.Tensor, k, mesh: Mesh, quad_order: int, mode: str = "table",
         tables: Tables = None, dtype=torch.complex64) -> torch.Tensor:
    """Differentiable fill: gradients flow to V (vertices) and k (a tensor)."""
    kk = k if isinstance(k, torch.Tensor) else torch.tensor(float(k), dtype=torch.float64)
    return _FillFn.apply(V, kk, mesh, quad_order, mode, tables, dtype)
