"""CPU oracle for frequent-episode counting -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_0905_2200_amd``) and never imports it.

Contents
--------
* ``fe_oracle.c`` (built to ``liboracle.so``): the paper's serial counters,
  Algorithm 1 (Sec. 5.1, full timestamp lists, exact ``(lo, hi]`` test) and
  Algorithm 3 (Sec. 5.3.1, one timestamp per node, relaxed ``[0, hi]`` test),
  plus Algorithm 4 (Sec. 5.3.2, two-pass elimination).
* :mod:`oracle.brute`: brute force from the definition (Sec. 2: occurrences
  and the largest set of non-overlapped occurrences) for tiny streams.
* :mod:`oracle.mine`: level-wise mining for Problem 1 (Sec. 2) with its own
  candidate generator (Sec. 3 / Sec. 5 describe the level-wise scheme).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fe_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODE_EXACT = 0          # Algorithm 1, (lo, hi]
MODE_RELAXED = 1        # Algorithm 3, [0, hi], latest timestamp only
MODE_RELAXED_LISTS = 2  # Algorithm 1's full lists with the [0, hi] test

NMAX = 8


def build(force: bool = False) -> str:
    """Compile fe_oracle.c with gcc into liboracle.so (in place)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.orc_count_many.argtypes = [P, P, i64, i32, P, P, P, P, i64, i32, i32, i32, i32, P]
        L.orc_count_many.restype = ctypes.c_int
        L.orc_two_pass.argtypes = [P, P, i64, i32, P, P, P, P, i64, i32, i64, i32, i32, P, P]
        L.orc_two_pass.restype = i64
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def pack_candidates(episodes):
    """Pack a list of episodes into the row-major candidate table.

    Each episode is ``(types, lo, hi)`` with ``len(lo) == len(hi) ==
    len(types) - 1``.  Returns ``(types[M, nmax], len[M], lo[M, nmax-1],
    hi[M, nmax-1], nmax)`` with unused entries set to -1 (types) / 0.
    """
    M = len(episodes)
    nmax = max([len(e[0]) for e in episodes] + [1])
    T = np.full((M, nmax), -1, np.int32)
    Ln = np.zeros(M, np.int32)
    LO = np.zeros((M, max(nmax - 1, 0)), np.int32)
    HI = np.zeros((M, max(nmax - 1, 0)), np.int32)
    for m, (ty, lo, hi) in enumerate(episodes):
        N = len(ty)
        assert len(lo) == N - 1 and len(hi) == N - 1
        T[m, :N] = ty
        Ln[m] = N
        if N > 1:
            LO[m, :N - 1] = lo
            HI[m, :N - 1] = hi
    return T, Ln, LO, HI, nmax


def count(ids, ticks, num_types, types, lens, lo, hi, mode=MODE_EXACT,
          projection=False, nthreads=0):
    """Count every candidate of a packed table; returns int64[M]."""
    ids, ticks = _i32(ids), _i32(ticks)
    types = _i32(types)
    M = types.shape[0]
    nmax = types.shape[1] if types.ndim == 2 else 1
    lens = _i32(lens)
    lo = _i32(lo).reshape(M, max(nmax - 1, 0)) if M else np.zeros((0, max(nmax - 1, 0)), np.int32)
    hi = _i32(hi).reshape(M, max(nmax - 1, 0)) if M else np.zeros((0, max(nmax - 1, 0)), np.int32)
    lo, hi = np.ascontiguousarray(lo), np.ascontiguousarray(hi)
    out = np.zeros(max(M, 1), np.int64)
    rc = lib().orc_count_many(_ptr(ids), _ptr(ticks), len(ids), int(num_types),
                              _ptr(types), _ptr(lens), _ptr(lo), _ptr(hi), M,
                              nmax, int(mode), int(bool(projection)), int(nthreads),
                              _ptr(out))
    if rc != 0:
        raise ValueError("oracle count failed (bad input or out of memory)")
    return out[:M]


def count_episodes(ids, ticks, episodes, mode=MODE_EXACT, num_types=None,
                   projection=False, nthreads=0):
    """Convenience: count a python list of ``(types, lo, hi)`` episodes."""
    T, Ln, LO, HI, _ = pack_candidates(episodes)
    if num_types is None:
        num_types = int(max([int(np.max(ids)) + 1 if len(ids) else 1] +
                            [int(max(e[0])) + 1 for e in episodes]))
    return count(ids, ticks, num_types, T, Ln, LO, HI, mode, projection, nthreads)


def two_pass(ids, ticks, num_types, types, lens, lo, hi, theta,
             projection=False, nthreads=0):
    """Algorithm 4: returns (upper int64[M], exact int64[M] with -1 = pruned)."""
    ids, ticks = _i32(ids), _i32(ticks)
    types = _i32(types)
    M = types.shape[0]
    nmax = types.shape[1]
    lens = _i32(lens)
    lo = np.ascontiguousarray(_i32(lo).reshape(M, max(nmax - 1, 0)))
    hi = np.ascontiguousarray(_i32(hi).reshape(M, max(nmax - 1, 0)))
    up = np.zeros(max(M, 1), np.int64)
    ex = np.zeros(max(M, 1), np.int64)
    ns = lib().orc_two_pass(_ptr(ids), _ptr(ticks), len(ids), int(num_types),
                            _ptr(types), _ptr(lens), _ptr(lo), _ptr(hi), M, nmax,
                            int(theta), int(bool(projection)), int(nthreads),
                            _ptr(up), _ptr(ex))
    if ns < 0:
        raise ValueError("oracle two-pass failed")
    return up[:M], ex[:M]
