"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two legs, each in a child process with the sanitizer runtime preloaded:
  * the oracle (oracle.c) rebuilt by gcc with -fsanitize=address,undefined and
    driven through a small end-to-end run: rule, edges, distance range, both
    tables, touching and regular entries in table and direct mode, the
    triangle-pair row fill, the MFIE and the angular inner integrals;
  * the host translation units of the library (api.cpp, tune.cpp: mesh
    analysis, tile and triangle-block plans, touching-pair lists, near-field
    patterns, workspace sizing and argument checking) rebuilt by hipcc with
    host-only sanitizers and linked against the in-tree objects of the HIP
    sources; no GPU call is made.
Each child prints its results as JSON; they must equal the uninstrumented
builds' results, and any sanitizer report fails the test.
"""

import glob
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1901_04162_amd import meshes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1901_04162_amd", "csrc")
OBJ = os.path.join(ROOT, "paper_1901_04162_amd", "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_OBJS = ["geometry.o", "tables.o", "fill.o", "backward.o", "scatter.o", "mfie.o", "angular.o"]
SAN_ENV = {
    "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:detect_odr_violation=0",
    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
}


def _run_child(code, env_extra, preload):
    env = dict(os.environ, **SAN_ENV, **env_extra)
    env["LD_PRELOAD"] = preload
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=600, cwd=ROOT)
    err = r.stderr
    assert "AddressSanitizer" not in err and "runtime error" not in err, err[-4000:]
    assert r.returncode == 0, err[-4000:]
    line = [s for s in r.stdout.splitlines() if s.startswith("{")][-1]
    return json.loads(line)


def _flat(v):
    if not isinstance(v, list):
        return np.array([v], dtype=float)
    return np.concatenate([_flat(y) for y in v]) if v else np.zeros(0)


ORACLE_RUN = r"""
import json, os, sys
import numpy as np
import oracle
assert oracle._SO == os.environ.get("MOMFILL_ORACLE_SO", oracle._SO)
from paper_1901_04162_amd import meshes

def c(z):
    z = np.asarray(z)
    return [float(np.real(z).sum()), float(np.imag(z).sum()), float(np.abs(z).sum())]

V, F = meshes.icosphere(1)
E = oracle.rwg(V, F)
k, Q = 3.0, 6
lo, hi = oracle.r_range(V, F, Q)
g = oracle.build_table(oracle.GREEN, k, lo, hi, 1e-6)
x = oracle.build_table(oracle.EXP, k, 0.0, hi, 1e-6)
rr = np.linspace(lo, hi, 57)
out = {
    "rule": c(oracle.quad_rule(Q)[1]),
    "edges": int(E.astype(np.int64).sum()),
    "range": [lo, hi],
    "green": [g.n, g.m, c(g(rr))],
    "exp": [x.n, x.m, c(x(rr))],
    "direct": c(oracle.fill(V, F, k, Q)),
    "table": c(oracle.fill(V, F, k, Q, mode=oracle.TABLE, gtable=g)),
    "rows": c(oracle.fill_rows(V, F, E, k, Q, 3, 11)),
    "mfie": c(oracle.mfie_entries(V, F, E, k, Q, np.arange(40), np.arange(40)[::-1])),
    "angular": c(oracle.angular_entries(V, F, E, k, Q, 4, np.arange(30), np.arange(30) % 7)),
    "pot": list(oracle.tri_potentials(V[F[0, 0]], V[F[0, 1]], V[F[0, 2]], V[F[5, 0]])[1]),
}
print(json.dumps(out))
"""


def test_oracle_under_asan_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    so = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                    "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    os.path.join(ROOT, "oracle", "oracle.c"), "-o", so, "-lm"], check=True)
    san = _run_child(ORACLE_RUN, {"MOMFILL_ORACLE_SO": so, "OMP_NUM_THREADS": "2"}, asan)
    ref = _run_child(ORACLE_RUN, {"OMP_NUM_THREADS": "2"}, "")
    assert san.keys() == ref.keys()
    for key in ref:
        np.testing.assert_allclose(_flat(san[key]), _flat(ref[key]), rtol=1e-12, atol=1e-14,
                                   err_msg=key)


LIB_RUN = r"""
import ctypes as C, json
import numpy as np
import paper_1901_04162_amd as mf
from paper_1901_04162_amd import meshes

import os
L = mf.lib()
assert mf._lib.SO_PATH == os.environ.get("MOMFILL_SO", mf._lib.SO_PATH)
out = {}
for name, (V, F) in {"ico1": meshes.icosphere(1), "ico3": meshes.icosphere(3),
                     "plate": meshes.plate(24)}.items():
    m = mf.Mesh(F, V.shape[0])
    E = m.edges()
    n = C.c_size_t()
    assert L.mf_mesh_workspace_bytes(m.handle, C.byref(n)) == 0
    nf = mf.NearField(m, V, 0.3)
    rp, col = nf.pattern()
    t = C.c_size_t()
    assert L.mf_near_workspace_bytes(nf._h, C.byref(t)) == 0
    out[name] = [m.n_edges, int(E.astype(np.int64).sum()), m.n_touching(), list(m.plan()),
                 list(m.tb_plan()), int(n.value), nf.nnz, nf.n_tiles,
                 int(rp.astype(np.int64).sum()), int(col.astype(np.int64).sum()), int(t.value)]
for F in ([[0, 1, 2], [1, 0, 3], [0, 1, 4]], [[0, 1, 2], [0, 1, 3]], [[0, 0, 2], [0, 2, 3]],
          [[0, 1, 9], [1, 0, 3]], [[0, 1, 2]]):
    try:
        mf.Mesh(np.array(F), 5)
        raise SystemExit("bad mesh accepted")
    except mf.MomfillError as e:
        assert e.code == mf._lib.MF_EMESH
V, F = meshes.icosphere(2)
m = mf.Mesh(F, V.shape[0])
z, h = C.c_void_p(1), C.c_void_p()
assert L.mf_fill_Z(m.handle, z, 1.0, 5, 1, None, z, 0, m.n_edges, None) == mf._lib.MF_EINVAL
assert L.mf_fill_Z(m.handle, z, 1.0, 3, 1, None, z, 0, m.n_edges - 1, None) == mf._lib.MF_EINVAL
assert L.mf_build_tables(-1.0, 0.1, 1.0, 1e-6, z, 1 << 20, C.byref(h), None) == mf._lib.MF_EINVAL
tb = []
for tol in (1e-4, 1e-6):
    t = C.c_size_t()
    assert L.mf_tables_workspace_bytes(17.0, 0.0331, 1.9998, tol, C.byref(t)) == 0
    tb.append(int(t.value))
arr = (C.c_void_p * 2)(m.handle.value, m.handle.value)
t = C.c_size_t()
assert L.mf_batch_workspace_bytes(2, arr, C.byref(t)) == 0
out["tables"] = tb
out["batch"] = int(t.value)
print(json.dumps(out))
"""


def test_library_host_code_under_asan_ubsan(tmp_path):
    rts = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    objs = [os.path.join(OBJ, o) for o in HIP_OBJS]
    if not rts or not os.path.exists(HIPCC):
        pytest.skip("hipcc or clang's AddressSanitizer runtime is not installed")
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("in-tree HIP objects missing: run the library build first")
    # host-only instrumentation: every -fsanitize= goes to the host pass
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined"]
    own = []
    for src in ("api.cpp", "tune.cpp"):
        o = str(tmp_path / (src + ".o"))
        subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer", *san,
                        "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-c",
                        os.path.join(CSRC, src), "-o", o], check=True, capture_output=True)
        own.append(o)
    so = str(tmp_path / "libmomfill_san.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *san, *own, *objs, "-o",
                    so], check=True, capture_output=True)
    undef = subprocess.run(["nm", "-D", "--undefined-only", so], capture_output=True,
                           text=True).stdout
    assert "__asan_report" in undef and "__ubsan_handle" in undef  # instrumented
    got = _run_child(LIB_RUN, {"MOMFILL_SO": so}, rts[0])
    ref = _run_child(LIB_RUN, {}, "")
    assert got == ref
