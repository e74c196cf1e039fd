"""Neighborhoods n_i of Sec. II.A by brute force -- oracle side.

Test infrastructure only (see ``oracle/__init__.py``).

``neighbors`` calls the plain C triple loop in ``nbrs.c`` (built by
``build_c``); ``neighbors_py`` is the same definition in pure Python for tiny
inputs, used to pin the C version.  Both return ``oracle.mtp.Pairs`` sorted
by (i, j, shift).
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess

import numpy as np

from .mtp import Pairs

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_liboracle_nbrs.so")
_lib = None


def build_c(force=True):
    """Compile nbrs.c with gcc (OpenMP) next to this file."""
    if force or not os.path.exists(_SO):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _SO,
                               os.path.join(_HERE, "nbrs.c"), "-lm"])


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_c(force=True)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        lib.oracle_nbr_count.restype = ctypes.c_int64
        lib.oracle_nbr_count.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double, P]
        lib.oracle_nbr_fill.restype = None
        lib.oracle_nbr_fill.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double, P, P, P]
        lib.oracle_nbr_count_sel.restype = ctypes.c_int64
        lib.oracle_nbr_count_sel.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double,
                                             ctypes.c_int64, P, P]
        lib.oracle_nbr_fill_sel.restype = None
        lib.oracle_nbr_fill_sel.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double,
                                            ctypes.c_int64, P, P, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def neighbors(pos, cell, pbc, r_cut, atoms=None):
    """All (i, j, n) with 0 < |x_j + n H - x_i| < r_cut (Sec. II.A).

    atoms: optional subset of central atoms (then ``Pairs.i`` holds the
    original atom indices).
    """
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    cell = np.ascontiguousarray(cell, dtype=np.float64)
    pbc_a = np.ascontiguousarray([1 if p else 0 for p in pbc], dtype=np.int32)
    n = len(pos)
    if atoms is None:
        counts = np.zeros(n, dtype=np.int64)
        total = lib.oracle_nbr_count(n, _ptr(pos), _ptr(cell), _ptr(pbc_a), r_cut, _ptr(counts))
        off = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(counts, out=off[1:])
        j = np.zeros(total, dtype=np.int32)
        sh = np.zeros((total, 3), dtype=np.int32)
        lib.oracle_nbr_fill(n, _ptr(pos), _ptr(cell), _ptr(pbc_a), r_cut, _ptr(off), _ptr(j), _ptr(sh))
        i = np.repeat(np.arange(n, dtype=np.int64), counts)
    else:
        sel = np.ascontiguousarray(atoms, dtype=np.int64)
        counts = np.zeros(len(sel), dtype=np.int64)
        total = lib.oracle_nbr_count_sel(n, _ptr(pos), _ptr(cell), _ptr(pbc_a), r_cut, len(sel),
                                         _ptr(sel), _ptr(counts))
        off = np.zeros(len(sel) + 1, dtype=np.int64)
        np.cumsum(counts, out=off[1:])
        j = np.zeros(total, dtype=np.int32)
        sh = np.zeros((total, 3), dtype=np.int32)
        lib.oracle_nbr_fill_sel(n, _ptr(pos), _ptr(cell), _ptr(pbc_a), r_cut, len(sel), _ptr(sel),
                                _ptr(off), _ptr(j), _ptr(sh))
        i = np.repeat(sel, counts)
    return Pairs(i.astype(np.int64), j.astype(np.int64), sh.astype(np.int64))


def neighbors_py(pos, cell, pbc, r_cut):
    """The same definition as ``neighbors`` in plain Python (tiny inputs)."""
    pos = np.asarray(pos, dtype=np.float64)
    H = np.asarray(cell, dtype=np.float64)
    Hi = np.linalg.inv(H)
    s = pos @ Hi
    vol = abs(np.linalg.det(H))
    h = [vol / np.linalg.norm(np.cross(H[(k + 1) % 3], H[(k + 2) % 3])) for k in range(3)]
    out = []
    for i in range(len(pos)):
        for j in range(len(pos)):
            rng = []
            for k in range(3):
                if pbc[k]:
                    d = s[j, k] - s[i, k]
                    rng.append(range(math.floor(-d - r_cut / h[k]) - 1, math.ceil(-d + r_cut / h[k]) + 2))
                else:
                    rng.append(range(0, 1))
            for n in itertools.product(*rng):
                if i == j and n == (0, 0, 0):
                    continue
                r = pos[j] + np.asarray(n) @ H - pos[i]
                if np.linalg.norm(r) < r_cut:
                    out.append((i, j) + tuple(n))
    out.sort()
    a = np.asarray(out, dtype=np.int64).reshape(-1, 5)
    return Pairs(a[:, 0], a[:, 1], a[:, 2:5])
