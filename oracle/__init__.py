"""Python access to the sequential CPU oracle (polylla_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this module; the product package never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "polylla_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORC_OK, ORC_EINVAL, ORC_ERANGE, ORC_EDEGEN, ORC_ENONMANIFOLD, ORC_ENOMEM, ORC_ECORRUPT = (
    0, -1, -2, -3, -4, -5, -10)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle returned {code}")
        self.code = code


class _Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "nt", "nv", "nh", "nflipped", "nties", "nterminal", "ntips", "nmiddle",
        "npoly", "nloop_he")] + [(n, ctypes.c_double) for n in (
            "ms_build", "ms_label", "ms_repair", "ms_traverse", "ms_canon")]


def build_library(force: bool = True) -> str:
    """Compiles liboracle.so next to its source (plain C, -O3)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_NATIVE = os.path.join(_HERE, "liboracle_native.so")


def build_native_library() -> str:
    """Compiles liboracle_native.so for the host it runs on (-O3
    -march=native): the CPU baseline's build, made on the machine that times
    it.  The tests use the portable build."""
    tmp = _NATIVE + f".{os.getpid()}.tmp"
    subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                           "-o", tmp, _SRC])
    os.replace(tmp, _NATIVE)
    return _NATIVE


_lib = None
_lib_path = None


def use_library(path: str) -> None:
    """Makes every later oracle call in this process use the library at path
    (built from the same source)."""
    global _lib, _lib_path
    _lib, _lib_path = None, path


def _load():
    global _lib
    if _lib is None:
        path = _lib_path or _LIB
        if path == _LIB and not os.path.exists(_LIB):
            build_library()
        lib = ctypes.CDLL(path)
        p32 = ctypes.POINTER(ctypes.c_int32)
        p8 = ctypes.POINTER(ctypes.c_uint8)
        lib.orc_polylla.argtypes = [p32, ctypes.c_int32, p32, ctypes.c_int32,
                                    p32, p32, p32, p32, p32, p32, p32, p8, p8, p8,
                                    ctypes.POINTER(_Stats)]
        lib.orc_polylla.restype = ctypes.c_int
        lib.orc_build.argtypes = [p32, ctypes.c_int32, p32, ctypes.c_int32, p32, p32,
                                  ctypes.POINTER(_Stats)]
        lib.orc_build.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a, ty=ctypes.c_int32):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ty))


@dataclass
class OracleResult:
    org: np.ndarray
    twin: np.ndarray
    next: np.ndarray
    prev: np.ndarray
    seeds: np.ndarray
    loop_off: np.ndarray
    loop_he: np.ndarray
    longest: np.ndarray      # uint8 per half-edge: longest edge of its triangle
    frontier: np.ndarray     # uint8 per half-edge: label-phase frontier
    frontier_rep: np.ndarray  # uint8 per half-edge: frontier after the repair
    stats: dict


def _inputs(xy, tri):
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.int32).reshape(-1, 2))
    tri = np.ascontiguousarray(np.asarray(tri, dtype=np.int32).reshape(-1, 3))
    return xy, tri


def polylla(xy, tri) -> OracleResult:
    """Runs the oracle; raises OracleError on an input the pipeline rejects."""
    xy, tri = _inputs(xy, tri)
    nv, nt = xy.shape[0], tri.shape[0]
    nh = 3 * nt
    org = np.empty(nh, np.int32)
    twin = np.empty(nh, np.int32)
    nx = np.empty(nh, np.int32)
    pv = np.empty(nh, np.int32)
    seeds = np.empty(max(nt, 1), np.int32)
    loop_off = np.empty(nt + 1, np.int32)
    loop_he = np.empty(max(nh, 1), np.int32)
    lg = np.empty(max(nh, 1), np.uint8)
    fr = np.empty(max(nh, 1), np.uint8)
    fr2 = np.empty(max(nh, 1), np.uint8)
    st = _Stats()
    rc = _load().orc_polylla(_ptr(xy), nv, _ptr(tri), nt, _ptr(org), _ptr(twin), _ptr(nx), _ptr(pv),
                             _ptr(seeds), _ptr(loop_off), _ptr(loop_he), _ptr(lg, ctypes.c_uint8),
                             _ptr(fr, ctypes.c_uint8), _ptr(fr2, ctypes.c_uint8), ctypes.byref(st))
    if rc != ORC_OK:
        raise OracleError(rc)
    stats = {n: getattr(st, n) for n, _ in _Stats._fields_}
    p, f = int(st.npoly), int(st.nloop_he)
    return OracleResult(org, twin, nx, pv, seeds[:p].copy(), loop_off[:p + 1].copy(),
                        loop_he[:f].copy(), lg[:nh], fr[:nh], fr2[:nh], stats)


def build(xy, tri):
    """Half-edge structure only: (org, twin, stats)."""
    xy, tri = _inputs(xy, tri)
    nv, nt = xy.shape[0], tri.shape[0]
    org = np.empty(3 * nt, np.int32)
    twin = np.empty(3 * nt, np.int32)
    st = _Stats()
    rc = _load().orc_build(_ptr(xy), nv, _ptr(tri), nt, _ptr(org), _ptr(twin), ctypes.byref(st))
    if rc != ORC_OK:
        raise OracleError(rc)
    return org, twin, {n: getattr(st, n) for n, _ in _Stats._fields_}
