"""ctypes front end of the C oracle fill (oracle/csrc/efie_oracle.c).

Same definition as efie.fill; used where the numpy version is too slow
(full matrices beyond a few hundred unknowns, the CPU timing baseline).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .efie import Geometry
from .mesh import flagged_pairs

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "efie_oracle.c")
_LIB = os.path.join(_HERE, "_efie_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p; I64 = ctypes.c_int64
        lib.oracle_fill.argtypes = [I64, I64, ctypes.c_int, P, P, P, P, P, P, P, P,
                                    ctypes.c_double, I64, P, P, P]
        lib.oracle_fill.restype = None
        lib.oracle_k0k1.argtypes = [I64, P, P, P, P]
        lib.oracle_k0k1.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def colour_triangles(m_of: np.ndarray) -> list[np.ndarray]:
    """Greedy colouring of triangles so that no two triangles of one colour share an RWG."""
    F = m_of.shape[0]
    owners: dict[int, list[int]] = {}
    for t in range(F):
        for m in m_of[t]:
            owners.setdefault(int(m), []).append(t)
    colour = -np.ones(F, np.int64)
    for t in range(F):
        used = {colour[o] for m in m_of[t] for o in owners[int(m)] if o != t and colour[o] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[t] = c
    return [np.nonzero(colour == c)[0] for c in range(colour.max() + 1)]


def fill(rwg: dict, k: float, rule=None, near_factor: float = 2.0, singular: bool = True) -> np.ndarray:
    lib = _load()
    G = Geometry(rwg, rule)
    F, N = rwg["F"], rwg["N"]
    if singular:
        flags = flagged_pairs(rwg, near_factor).astype(np.uint8)
    else:
        flags = np.zeros((F, F), np.uint8)
    cols = colour_triangles(G.m_of)
    ptr = np.zeros(len(cols) + 1, np.int64)
    ptr[1:] = np.cumsum([c.size for c in cols])
    tris = np.ascontiguousarray(np.concatenate(cols).astype(np.int64))
    X = np.ascontiguousarray(G.X); Vf = np.ascontiguousarray(G.Vf); tri = np.ascontiguousarray(G.tri)
    w = np.ascontiguousarray(G.w); area = np.ascontiguousarray(rwg["area"])
    m_of = np.ascontiguousarray(G.m_of.astype(np.int64)); s_of = np.ascontiguousarray(G.s_of)
    Z = np.zeros((N, N), np.complex128)
    lib.oracle_fill(F, N, int(w.size), _ptr(w), _ptr(X), _ptr(Vf), _ptr(tri), _ptr(area),
                    _ptr(m_of), _ptr(s_of), _ptr(flags), float(k), len(cols), _ptr(ptr), _ptr(tris), _ptr(Z))
    return Z


def k0_k1(x: np.ndarray, tri: np.ndarray):
    lib = _load()
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.float64)
    K0 = np.zeros(x.shape[0]); K1 = np.zeros((x.shape[0], 3))
    lib.oracle_k0k1(x.shape[0], _ptr(x), _ptr(tri), _ptr(K0), _ptr(K1))
    return K0, K1
