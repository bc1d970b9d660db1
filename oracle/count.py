"""Python side of the simulated-execution count oracle (count_oracle.c).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "count_oracle.c")
_SO = os.path.join(_HERE, "_count_oracle.so")

FAMILIES = {"stream": 0, "lds": 1, "fma": 2, "rsqrt": 3, "barrier": 4,
            "empty": 5, "matmul": 6, "transpose": 7, "stencil": 8,
            "nbody": 9, "arith": 10, "conv": 11}
OPS = {
    "stream": {"load": 0, "store": 1, "copy": 2, "add4": 3, "filled": 4,
               "axpby": 5},
    "arith": {"div": 0, "exp": 1},
    "lds": {"read": 0, "write": 1},
    "matmul": {"tiled": 0, "naive": 1},
    "transpose": {"tiled": 0, "naive_wc": 1, "naive_rc": 2},
}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into oracle/_count_oracle.so."""
    if force or not os.path.exists(_SO) or \
            os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        L.oracle_nout.restype = ctypes.c_int
        L.oracle_name.argtypes = [ctypes.c_int, ctypes.c_char_p, ctypes.c_int]
        L.oracle_count.argtypes = [ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int64),
                                   ctypes.c_char_p, ctypes.c_int]
        L.oracle_classify_1d.argtypes = [
            ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
            ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        for nm, ct in (("oracle_fma_chain_f32", ctypes.c_float),
                       ("oracle_fma_chain_f64", ctypes.c_double)):
            getattr(L, nm).argtypes = [ctypes.POINTER(ct), ctypes.POINTER(ct),
                                       ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int64]
        _lib = L
    return _lib


_names = None


def names():
    global _names
    if _names is None:
        L = lib()
        buf = ctypes.create_string_buffer(64)
        out = []
        for i in range(L.oracle_nout()):
            L.oracle_name(i, buf, 64)
            out.append(buf.value.decode())
        _names = out
    return _names


CLASS_NAMES = ["0", "1", "1/2", "2/2", "1/3", "2/3", "3/3", "1/4", "2/4",
               "3/4", "4/4", "1/>4", "2/>4", "3/>4", "4/>4"]


def params(v: dict) -> list:
    """Pack a variant dict into the oracle's 16 int64 parameters."""
    fam = v["family"]
    eb = 8 if v.get("dtype", "f32") == "f64" else 4
    op = OPS.get(fam, {}).get(v.get("op"), 0)
    n = v.get("n", 0)
    wgx = v.get("wg", v.get("wx", v.get("T", 0)))
    wgy = v.get("wy", 1)
    reps = {"stream": v.get("U", 1), "lds": v.get("R", 0),
            "fma": v.get("F", 0), "rsqrt": v.get("F", 0), "arith": v.get("F", 0),
            "barrier": v.get("B", 0)}.get(fam, 0)
    K = v.get("K", 1)
    if fam == "stream" and v.get("op") == "filled":
        K = v.get("c", v["s"])  # cells read of every s
    return [FAMILIES[fam], eb, op, n, v.get("m", 0), v.get("l", 0), wgx, wgy,
            v.get("T", 0), v.get("s", v.get("b", 1)), v.get("gs", 1),
            v.get("vec", 1), reps, K, v.get("W", 0), v.get("groups", 0)]


def count(v: dict, with_footprints: bool = False) -> dict:
    """Simulated-execution counts of one variant as {name: int}.  Zero
    entries are dropped; `with_footprints` keeps the per-array |F| and
    |Fill| diagnostics ("foot.F.<a>", "foot.fill.<a>")."""
    L = lib()
    nout = L.oracle_nout()
    p = (ctypes.c_int64 * 16)(*params(v))
    out = (ctypes.c_int64 * nout)()
    msg = ctypes.create_string_buffer(256)
    if L.oracle_count(p, out, msg, 256) != 0:
        raise ValueError("oracle: " + msg.value.decode())
    res = {}
    for nm, x in zip(names(), out):
        if x and (with_footprints or not nm.startswith("foot.")):
            res[nm] = int(x)
    return res


def classify_1d(cells: int, n: int, sites, elem: int = 4, vec: int = 1):
    """Stride class names of 1-D access sites [(coef, offset), ...] over
    i in [0, n) on one array of `cells` cells."""
    L = lib()
    k = len(sites)
    coef = (ctypes.c_int64 * k)(*[s[0] for s in sites])
    off = (ctypes.c_int64 * k)(*[s[1] for s in sites])
    cls = (ctypes.c_int * k)()
    if L.oracle_classify_1d(cells, n, k, coef, off, elem, vec, cls) != 0:
        raise ValueError("oracle: bad access list")
    return [CLASS_NAMES[c] for c in cls]
