"""Python front end of the plain-C line oracle (oracle/field_lines.c).

TEST INFRASTRUCTURE ONLY.  Builds field_lines.c with gcc (-O2, OpenMP) into
oracle/_build/ and evaluates exact FP64 z-lines of a box of any size, for
sampled parity where a full FP64 box does not fit in host memory.
"""
import ctypes
import os
import subprocess

import numpy as np

from .field import COMPONENTS

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "field_lines.c")
_OUT = os.path.join(_HERE, "_build", "liboracle_lines.so")
_lib = None


def build(force=False):
    """Compile the C oracle (gcc -O2 -fopenmp -shared)."""
    os.makedirs(os.path.dirname(_OUT), exist_ok=True)
    if force or not os.path.exists(_OUT) or \
            os.path.getmtime(_OUT) < os.path.getmtime(_SRC):
        tmp = _OUT + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _OUT)
    return _OUT


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        f = _lib.oracle_field_lines
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_double,
                      ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_long,
                      ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_int]
    return _lib


def field_lines(n, seed, table, columns, comps=("delta", "zz"), f=1.0,
                fixed_amp=False, only_n2=-1, nthreads=None):
    """Exact lines C(mx, my, :) for each (mx, my) in columns.

    Returns (re, im), each of shape [len(columns), n]: component comps[0] and
    component comps[1] (zero if comps has one entry)."""
    lib = _load()
    if nthreads is None:
        nthreads = max(1, min(16, os.cpu_count() or 1))
    cols = np.asarray(columns, dtype=np.int32).reshape(-1, 2)
    mx = np.ascontiguousarray(cols[:, 0])
    my = np.ascontiguousarray(cols[:, 1])
    tab = np.ascontiguousarray(table, dtype=np.float64)
    assert tab.shape[0] >= 3 * (n // 2) ** 2 + 1
    re = np.zeros((len(cols), n))
    im = np.zeros((len(cols), n))
    ca = COMPONENTS.index(comps[0])
    cb = COMPONENTS.index(comps[1]) if len(comps) > 1 else -1
    rc = lib.oracle_field_lines(int(n), int(seed), float(f), ca, cb,
                                int(bool(fixed_amp)), int(only_n2),
                                tab.ctypes.data, len(cols), mx.ctypes.data,
                                my.ctypes.data, re.ctypes.data, im.ctypes.data,
                                int(nthreads))
    if rc != 0:
        raise MemoryError("oracle_field_lines failed")
    return re, im
