"""Pin strength: plausible mistakes planted in a copy of the connection-scan
oracle (on the CPU, in a temporary directory) must be caught by the brute-force
pins.  Each mutant is one edit of csa.c; the test compiles it and compares it
with the state-closure brute force on tiny random timetables."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1912_00966_amd import synth

ORACLE_DIR = os.path.dirname(oracle.__file__)

MUTANTS = {
    "strict boarding test": ("tu <= h->t[i]", "tu < h->t[i]"),
    "duration dropped": ("int32_t a = h->t[i] + h->lam[i];", "int32_t a = h->t[i];"),
    "head and tail swapped": ("a < arr[h->v[i]]) arr[h->v[i]] = a;", "a < arr[h->u[i]]) arr[h->u[i]] = a;"),
    "scan starts after ts": ("if (h->t[mid] < ts)", "if (h->t[mid] <= ts)"),
    "source not initialised": ("arr[s] = ts;\n  /* first", "/* first"),
    "reverse time order": ("int64_t i = (int64_t)idx[k];", "int64_t i = (int64_t)idx[n - 1 - k];"),
    "high digit of the time not sorted": ("pass < 2; ++pass", "pass < 1; ++pass"),
    "boarding tests arrival of head": ("int32_t tu = arr[h->u[i]];", "int32_t tu = arr[h->v[i]];"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(os.path.join(ORACLE_DIR, "csa.c")).read()
    assert old in src, f"mutation site for '{name}' not found"
    d = tmp_path / name.replace(" ", "_")
    d.mkdir()
    shutil.copy(os.path.join(ORACLE_DIR, "oracle.h"), d / "oracle.h")
    (d / "csa.c").write_text(src.replace(old, new, 1))
    so = d / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(d / "csa.c")],
                   check=True)
    lib = ctypes.CDLL(str(so))
    p = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_csa_new.argtypes = [ctypes.c_int64, p, p, p, p, ctypes.c_int32]
    lib.oracle_csa_new.restype = ctypes.c_void_p
    lib.oracle_csa_query.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, p]
    lib.oracle_csa_free.argtypes = [ctypes.c_void_p]
    return lib


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    old, new = MUTANTS[name]
    lib = _build_mutant(tmp_path, name, old, new)
    p = ctypes.POINTER(ctypes.c_int32)
    rng = np.random.default_rng(2024)
    for k in range(3000):
        tt = synth.random_tiny(rng)
        s = int(rng.integers(0, tt.n_vertices))
        ts = int(rng.integers(0, 32))
        if k % 2:
            # the same timetable stretched over a wide time range: departure
            # times then differ in both 16-bit digits
            scale = 40_000
            tt = synth.Timetable("wide", tt.n_vertices, tt.u, tt.v, (tt.t * scale).astype(np.int32),
                                 (tt.lam * scale).astype(np.int32), -1, -1, -1)
            ts *= scale
        ref = oracle.brute_states(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, s, ts)
        arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (tt.u, tt.v, tt.t, tt.lam)]
        h = lib.oracle_csa_new(len(tt.u), *(a.ctypes.data_as(p) for a in arrs), tt.n_vertices)
        out = np.empty(tt.n_vertices, dtype=np.int32)
        lib.oracle_csa_query(h, s, ts, out.ctypes.data_as(p))
        lib.oracle_csa_free(h)
        if not np.array_equal(out, ref):
            return  # caught
    pytest.fail(f"mutant '{name}' survived 3000 brute-force comparisons")
