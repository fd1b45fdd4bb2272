"""gpolylla: Polylla polygonal meshing on MI355X through a C-ABI HIP library.

This module is argument marshalling only: every step of the pipeline runs in
the HIP kernels of libgpolylla.so (built in-tree by build_lib.py).  If the
library is missing the first call raises; there is no fallback.

The module-level functions carry the C names (gpolylla_ctx_create, ...); the
Context / Mesh / Result classes wrap them for convenience.  Inputs may be
numpy arrays (host) or torch tensors on the context's GPU (passed as device
pointers, read on the context's stream).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpolylla.so")

GP_OK = 0
GP_EINVAL, GP_ERANGE, GP_EDEGEN, GP_ENONMANIFOLD, GP_ENOMEM, GP_EHIP = -1, -2, -3, -4, -5, -6
GP_EAGAIN, GP_ETOOBIG, GP_ETIMEDOUT, GP_ECORRUPT = -7, -8, -9, -10
GP_IN_DEVICE = 0x1
GP_COMPACT = 0x8
GP_RENUMBER = 0x40
GP_ASYNC = 0x2
GP_GRAPH = 0x4
GP_OUT_LOOPS = 0x10
GP_OUT_NO_LOOPS = 0x20


class GPolyllaError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = gpolylla_strerror(code) if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")
        self.code = code


class gp_ctx_opts(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_size_t), ("stream", ctypes.c_void_p),
                ("profile", ctypes.c_int32), ("block", ctypes.c_int32), ("items", ctypes.c_int32)]


class gp_result_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("nt", "nv", "nh", "npoly", "nloop_he", "nterminal",
                                              "ntips", "nmiddle", "nties", "nflipped", "loops_only")]


class gp_serve_opts(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_size_t), ("max_batch", ctypes.c_int32),
                ("max_queue", ctypes.c_int32), ("n_lanes", ctypes.c_int32), ("loops_only", ctypes.c_int32)]


class gp_serve_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "rejected", "failed", "batches",
                                              "in_flight")] + \
               [(n, ctypes.c_double) for n in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "mtri_s")]


class gp_result_dev(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("next", "prev", "seeds", "loop_off", "loop_he")]


class gp_dev_counts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("status", "npoly", "nloop_he", "ntips", "nmiddle", "nties",
                                              "reserved0", "reserved1")]


GP_NOALLOC_SCRATCH_BYTES = 256 << 20


class gp_result_debug(ctypes.Structure):
    _fields_ = [("tflag_relink", ctypes.c_void_p), ("next_relink", ctypes.c_void_p),
                ("prev_relink", ctypes.c_void_p), ("tflag_final", ctypes.c_void_p), ("tips", ctypes.c_void_p),
                ("tips_cap", ctypes.c_int32), ("ntips", ctypes.c_int32)]


class gp_job(ctypes.Structure):
    _fields_ = [("xy", ctypes.c_void_p), ("nv", ctypes.c_int32), ("tri", ctypes.c_void_p), ("nt", ctypes.c_int32),
                ("next", ctypes.c_void_p), ("prev", ctypes.c_void_p), ("seeds", ctypes.c_void_p),
                ("loop_off", ctypes.c_void_p), ("loop_he", ctypes.c_void_p),
                ("npoly", ctypes.c_int32), ("nloop_he", ctypes.c_int32), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() or "
                           "python paper_2403_14723_amd/build_lib.py first")
    # torch ships its own HIP runtime with the same soname as ROCm's; loading
    # torch first makes the library bind to that one, so a process never holds
    # two HIP runtimes and torch tensors and streams are valid in the library
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "gpolylla_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "gpolylla_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(gp_ctx_opts), ctypes.POINTER(_P)]),
        "gpolylla_ctx_destroy": (None, [_P]),
        "gpolylla_ctx_pool_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t),
                                                   ctypes.POINTER(ctypes.c_size_t)]),
        "gpolylla_ctx_sync": (ctypes.c_int, [_P]),
        "gpolylla_ctx_kernel_ms": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_char_p),
                                                  ctypes.POINTER(ctypes.c_double),
                                                  ctypes.POINTER(ctypes.c_int64), ctypes.c_int]),
        "gpolylla_ctx_kernel_reset": (None, [_P]),
        "gpolylla_ctx_set_launch": (ctypes.c_int, [_P, ctypes.c_char_p]),
        "gpolylla_ctx_get_launch": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_int32]),
        "gpolylla_build_halfedges": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, ctypes.c_int32,
                                                    ctypes.c_uint32, ctypes.POINTER(_P)]),
        "gpolylla_mesh_copy": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(ctypes.c_int64)]),
        "gpolylla_mesh_size": (ctypes.c_int, [_P, _I32P, _I32P]),
        "gpolylla_mesh_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int64)]),
        "gpolylla_mesh_permutation": (ctypes.c_int, [_P, _P, _P]),
        "gpolylla_mesh_free": (None, [_P]),
        "gpolylla_mesh": (ctypes.c_int, [_P, _P, ctypes.c_uint32, ctypes.POINTER(_P)]),
        "gpolylla_mesh_batch": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_uint32,
                                               ctypes.POINTER(_P)]),
        "gpolylla_result_info": (ctypes.c_int, [_P, ctypes.POINTER(gp_result_info)]),
        "gpolylla_result_copy": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
        "gpolylla_result_device": (ctypes.c_int, [_P, ctypes.POINTER(gp_result_dev)]),
        "gpolylla_result_free": (None, [_P]),
        "gpolylla_mesh_noalloc": (ctypes.c_int, [_P, _P, ctypes.POINTER(gp_result_dev), _P]),
        "gpolylla_ctx_set_debug": (ctypes.c_int, [_P, ctypes.c_int32]),
        "gpolylla_result_debug": (ctypes.c_int, [_P, ctypes.POINTER(gp_result_debug)]),
        "gpolylla_mesh_jobs": (ctypes.c_int, [_P, ctypes.POINTER(gp_job), ctypes.c_int32, ctypes.c_int64,
                                              ctypes.c_uint32]),
        "gpolylla_serve_start": (ctypes.c_int, [_P, ctypes.POINTER(gp_serve_opts), ctypes.POINTER(_P)]),
        "gpolylla_serve_submit": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_uint64)]),
        "gpolylla_serve_submit_at": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_int64,
                                                    ctypes.POINTER(ctypes.c_uint64)]),
        "gpolylla_serve_wait": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(_P)]),
        "gpolylla_serve_stats": (ctypes.c_int, [_P, ctypes.POINTER(gp_serve_stats)]),
        "gpolylla_serve_reset_stats": (ctypes.c_int, [_P]),
        "gpolylla_serve_stop": (ctypes.c_int, [_P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def library():
    """The loaded ctypes library (raises when it has not been built)."""
    return _load()


def exported_symbols() -> list[str]:
    return [n for n in _SYMBOLS]


_SYMBOLS = ["gpolylla_strerror", "gpolylla_ctx_create", "gpolylla_ctx_destroy", "gpolylla_ctx_pool_bytes",
            "gpolylla_ctx_sync", "gpolylla_ctx_kernel_ms", "gpolylla_ctx_kernel_reset",
            "gpolylla_ctx_set_launch", "gpolylla_ctx_get_launch",
            "gpolylla_build_halfedges", "gpolylla_mesh_copy", "gpolylla_mesh_size", "gpolylla_mesh_bytes",
            "gpolylla_mesh_permutation",
            "gpolylla_mesh_free",
            "gpolylla_mesh", "gpolylla_mesh_batch", "gpolylla_result_info", "gpolylla_result_copy",
            "gpolylla_result_device", "gpolylla_result_free", "gpolylla_mesh_noalloc", "gpolylla_mesh_jobs",
            "gpolylla_ctx_set_debug", "gpolylla_result_debug",
            "gpolylla_serve_start", "gpolylla_serve_submit", "gpolylla_serve_submit_at",
            "gpolylla_serve_wait", "gpolylla_serve_stats", "gpolylla_serve_reset_stats", "gpolylla_serve_stop"]


def _check(rc: int, what: str):
    if rc != GP_OK:
        raise GPolyllaError(rc, what)


# ---------------------------------------------------------------------------
# C names
# ---------------------------------------------------------------------------

def gpolylla_strerror(code: int) -> str:
    return _load().gpolylla_strerror(code).decode()


def gpolylla_ctx_create(device: int = 0, opts: gp_ctx_opts | None = None):
    out = _P()
    _check(_load().gpolylla_ctx_create(device, ctypes.byref(opts) if opts else None, ctypes.byref(out)),
           "gpolylla_ctx_create")
    return out


def gpolylla_ctx_destroy(ctx):
    _load().gpolylla_ctx_destroy(ctx)


def gpolylla_ctx_sync(ctx):
    _check(_load().gpolylla_ctx_sync(ctx), "gpolylla_ctx_sync")


def gpolylla_ctx_kernel_ms(ctx) -> dict:
    cap = 16
    names = (ctypes.c_char_p * cap)()
    ms = (ctypes.c_double * cap)()
    cnt = (ctypes.c_int64 * cap)()
    n = _load().gpolylla_ctx_kernel_ms(ctx, names, ms, cnt, cap)
    return {names[i].decode(): (ms[i], int(cnt[i])) for i in range(n)}


def gpolylla_ctx_kernel_reset(ctx):
    _load().gpolylla_ctx_kernel_reset(ctx)


def gpolylla_ctx_set_launch(ctx, spec: str):
    _check(_load().gpolylla_ctx_set_launch(ctx, spec.encode()), f"gpolylla_ctx_set_launch({spec!r})")


def gpolylla_ctx_get_launch(ctx) -> str:
    lib = _load()
    n = lib.gpolylla_ctx_get_launch(ctx, None, 0)
    if n < 0:
        _check(n, "gpolylla_ctx_get_launch")
    buf = ctypes.create_string_buffer(n)
    _check(min(0, lib.gpolylla_ctx_get_launch(ctx, buf, n)), "gpolylla_ctx_get_launch")
    return buf.value.decode()


def gpolylla_ctx_pool_bytes(ctx) -> tuple[int, int]:
    held, used = ctypes.c_size_t(), ctypes.c_size_t()
    _check(_load().gpolylla_ctx_pool_bytes(ctx, ctypes.byref(held), ctypes.byref(used)), "pool_bytes")
    return held.value, used.value


def _as_input(a, dtype_cols, device=None):
    """Returns (pointer, count, keepalive, on_device).  A device tensor must
    be contiguous int32 of shape (n, dtype_cols) or (n * dtype_cols,), on
    `device` when that is given."""
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):
        if a.is_cuda:
            import torch
            if a.dtype != torch.int32 or not a.is_contiguous():
                raise ValueError("device inputs must be contiguous int32 tensors")
            if a.numel() % dtype_cols != 0 or (a.dim() >= 2 and (a.dim() > 2 or a.shape[-1] != dtype_cols)):
                raise ValueError(f"a device input of shape {tuple(a.shape)} is not (n, {dtype_cols})")
            if device is not None and a.device.index != device:
                raise ValueError(f"input on cuda:{a.device.index}, context on cuda:{device}")
            return ctypes.c_void_p(a.data_ptr()), a.numel() // dtype_cols, a, True
        a = a.numpy()
    arr = np.asarray(a, dtype=np.int32)
    if arr.size % dtype_cols != 0 or (arr.ndim >= 2 and (arr.ndim > 2 or arr.shape[-1] != dtype_cols)):
        raise ValueError(f"an input of shape {arr.shape} is not (n, {dtype_cols})")
    arr = np.ascontiguousarray(arr.reshape(-1, dtype_cols))
    return ctypes.c_void_p(arr.ctypes.data), arr.shape[0], arr, False


def gpolylla_build_halfedges(ctx, xy, tri, flags: int = 0, device=None):
    """device: the context's device, to check device tensors against."""
    pxy, nv, kxy, dxy = _as_input(xy, 2, device)
    ptri, nt, ktri, dtri = _as_input(tri, 3, device)
    if dxy != dtri:
        raise ValueError("xy and tri must both be host arrays or both device tensors")
    if dxy:
        flags |= GP_IN_DEVICE
    out = _P()
    _check(_load().gpolylla_build_halfedges(ctx, pxy, nv, ptri, nt, flags, ctypes.byref(out)),
           "gpolylla_build_halfedges")
    del kxy, ktri
    return out


def gpolylla_mesh(ctx, mesh, flags: int = 0):
    out = _P()
    _check(_load().gpolylla_mesh(ctx, mesh, flags, ctypes.byref(out)), "gpolylla_mesh")
    return out


def gpolylla_mesh_batch(ctx, meshes, flags: int = 0):
    n = len(meshes)
    arr = (_P * n)(*meshes)
    outs = (_P * n)()
    _check(_load().gpolylla_mesh_batch(ctx, arr, n, flags, outs), "gpolylla_mesh_batch")
    return [_P(o) for o in outs]


def gpolylla_mesh_copy(mesh):
    nv, nt = ctypes.c_int32(), ctypes.c_int32()
    _check(_load().gpolylla_mesh_size(mesh, ctypes.byref(nv), ctypes.byref(nt)), "gpolylla_mesh_size")
    org = np.empty(3 * nt.value, np.int32)
    twin = np.empty(3 * nt.value, np.int32)
    nflip = ctypes.c_int64()
    _check(_load().gpolylla_mesh_copy(mesh, org.ctypes.data, twin.ctypes.data, ctypes.byref(nflip)),
           "gpolylla_mesh_copy")
    return org, twin, int(nflip.value)


def gpolylla_mesh_free(mesh):
    _load().gpolylla_mesh_free(mesh)


def gpolylla_result_info(res) -> dict:
    info = gp_result_info()
    _check(_load().gpolylla_result_info(res, ctypes.byref(info)), "gpolylla_result_info")
    return {n: int(getattr(info, n)) for n, _ in gp_result_info._fields_}


def gpolylla_result_copy(res) -> dict:
    info = gpolylla_result_info(res)
    nh, p, f = info["nh"], info["npoly"], info["nloop_he"]
    out = {"seeds": np.empty(p, np.int32), "loop_off": np.empty(p + 1, np.int32), "loop_he": np.empty(f, np.int32)}
    if not info["loops_only"]:   # a loops-only served result holds no next'/prev'
        out["next"] = np.empty(nh, np.int32)
        out["prev"] = np.empty(nh, np.int32)
    ptr = {k: (v.ctypes.data if v.size else None) for k, v in out.items()}
    _check(_load().gpolylla_result_copy(res, ptr.get("next"), ptr.get("prev"), ptr["seeds"], ptr["loop_off"],
                                        ptr["loop_he"]), "gpolylla_result_copy")
    out["info"] = info
    return out


def gpolylla_result_device(res) -> dict:
    d = gp_result_dev()
    _check(_load().gpolylla_result_device(res, ctypes.byref(d)), "gpolylla_result_device")
    return {n: d.__getattribute__(n) for n, _ in gp_result_dev._fields_}


def gpolylla_result_free(res):
    _load().gpolylla_result_free(res)


def gpolylla_mesh_noalloc(ctx, mesh, out: gp_result_dev, counts_ptr: int) -> int:
    """Queues a meshing run into caller-allocated device buffers (out, and
    counts_ptr: device memory for a gp_dev_counts); returns the C status."""
    return _load().gpolylla_mesh_noalloc(ctx, mesh, ctypes.byref(out), ctypes.c_void_p(counts_ptr))


def gpolylla_mesh_jobs(ctx, jobs, group_triangles: int = 0, flags: int = 0) -> int:
    """Runs a ctypes array of gp_job (pointers filled in by the caller);
    returns the C status (every job's own status is in jobs[i].status)."""
    return _load().gpolylla_mesh_jobs(ctx, jobs, len(jobs), group_triangles, flags)


def gpolylla_serve_start(ctx, opts: gp_serve_opts | None = None):
    out = _P()
    _check(_load().gpolylla_serve_start(ctx, ctypes.byref(opts) if opts else None, ctypes.byref(out)),
           "gpolylla_serve_start")
    return out


def gpolylla_serve_submit(srv, xy, tri) -> int:
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.int32).reshape(-1, 2))
    tri = np.ascontiguousarray(np.asarray(tri, dtype=np.int32).reshape(-1, 3))
    t = ctypes.c_uint64()
    _check(_load().gpolylla_serve_submit(srv, xy.ctypes.data, xy.shape[0], tri.ctypes.data, tri.shape[0],
                                         ctypes.byref(t)), "gpolylla_serve_submit")
    return int(t.value)


def gpolylla_serve_submit_at(srv, xy, tri, arrival_ns: int) -> int:
    """Submits a request that arrived at arrival_ns (time.monotonic_ns())."""
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.int32).reshape(-1, 2))
    tri = np.ascontiguousarray(np.asarray(tri, dtype=np.int32).reshape(-1, 3))
    t = ctypes.c_uint64()
    _check(_load().gpolylla_serve_submit_at(srv, xy.ctypes.data, xy.shape[0], tri.ctypes.data, tri.shape[0],
                                            int(arrival_ns), ctypes.byref(t)), "gpolylla_serve_submit_at")
    return int(t.value)


def gpolylla_serve_wait(srv, ticket: int, timeout_ms: int = -1):
    out = _P()
    _check(_load().gpolylla_serve_wait(srv, ticket, timeout_ms, ctypes.byref(out)), "gpolylla_serve_wait")
    return out


def gpolylla_serve_stats(srv) -> dict:
    st = gp_serve_stats()
    _check(_load().gpolylla_serve_stats(srv, ctypes.byref(st)), "gpolylla_serve_stats")
    return {n: getattr(st, n) for n, _ in gp_serve_stats._fields_}


def gpolylla_serve_reset_stats(srv):
    _check(_load().gpolylla_serve_reset_stats(srv), "gpolylla_serve_reset_stats")


def gpolylla_serve_stop(srv):
    _check(_load().gpolylla_serve_stop(srv), "gpolylla_serve_stop")


# ---------------------------------------------------------------------------
# wrappers
# ---------------------------------------------------------------------------

class Mesh:
    def __init__(self, ctx: "Context", handle):
        self.ctx, self.handle = ctx, handle

    def copy(self):
        return gpolylla_mesh_copy(self.handle)

    def permutation(self) -> tuple:
        """(triangle new -> old, vertex new -> old) of a renumbered mesh"""
        nv, nt = ctypes.c_int32(), ctypes.c_int32()
        _check(_load().gpolylla_mesh_size(self.handle, ctypes.byref(nv), ctypes.byref(nt)), "gpolylla_mesh_size")
        tp = np.empty(max(nt.value, 1), np.int32)
        vp = np.empty(max(nv.value, 1), np.int32)
        _check(_load().gpolylla_mesh_permutation(self.handle, tp.ctypes.data, vp.ctypes.data),
               "gpolylla_mesh_permutation")
        return tp[:nt.value], vp[:nv.value]

    def nbytes(self) -> tuple[int, int]:
        """(device bytes the mesh holds, escaped values of a compact mesh)"""
        b, e = ctypes.c_size_t(), ctypes.c_int64()
        _check(_load().gpolylla_mesh_bytes(self.handle, ctypes.byref(b), ctypes.byref(e)), "gpolylla_mesh_bytes")
        return b.value, e.value

    def free(self):
        if self.handle:
            gpolylla_mesh_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            if self.handle and self.ctx.handle:
                self.free()
        except Exception:
            pass


def gpolylla_result_debug(res, nt: int) -> dict:
    """A debug run's intermediate stages of one result, as numpy arrays."""
    out = {"tflag_relink": np.zeros(max(nt, 1), np.uint8), "tflag_final": np.zeros(max(nt, 1), np.uint8),
           "next_relink": np.zeros(max(3 * nt, 1), np.int32), "prev_relink": np.zeros(max(3 * nt, 1), np.int32),
           "tips": np.zeros(max(nt, 1), np.int32)}
    d = gp_result_debug(*[out[k].ctypes.data for k in ("tflag_relink", "next_relink", "prev_relink",
                                                        "tflag_final", "tips")], len(out["tips"]), 0)
    _check(_load().gpolylla_result_debug(res, ctypes.byref(d)), "gpolylla_result_debug")
    for k in ("tflag_relink", "tflag_final"):
        out[k] = out[k][:nt]
    for k in ("next_relink", "prev_relink"):
        out[k] = out[k][:3 * nt]
    out["tips"] = np.sort(out["tips"][:min(d.ntips, len(out["tips"]))])
    out["ntips"] = d.ntips
    return out


class Result:
    def __init__(self, ctx: "Context", handle):
        self.ctx, self.handle = ctx, handle

    def info(self) -> dict:
        return gpolylla_result_info(self.handle)

    def copy(self) -> dict:
        return gpolylla_result_copy(self.handle)

    def debug(self) -> dict:
        """Intermediate stages (a run of a context with debug on)."""
        return gpolylla_result_debug(self.handle, self.info()["nt"])

    def device(self) -> dict:
        return gpolylla_result_device(self.handle)

    def free(self):
        if self.handle:
            gpolylla_result_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            if self.handle and self.ctx.handle:
                self.free()
        except Exception:
            pass


class Server:
    """Continuous-batching server (see gpolylla_serve_start)."""

    def __init__(self, ctx: "Context", pool_bytes: int = 0, max_batch: int = 0, max_queue: int = 0,
                 n_lanes: int = 0, loops_only: bool = False):
        """loops_only: results carry seeds and loops only (no next'/prev')."""
        self.handle = gpolylla_serve_start(ctx.handle, gp_serve_opts(pool_bytes, max_batch, max_queue, n_lanes,
                                                                     int(loops_only)))
        self._ctx = ctx

    def submit(self, xy, tri, arrival_ns: int = 0) -> int:
        """arrival_ns: when the request arrived (time.monotonic_ns()); its
        latency runs from then.  0: now."""
        if arrival_ns:
            return gpolylla_serve_submit_at(self.handle, xy, tri, arrival_ns)
        return gpolylla_serve_submit(self.handle, xy, tri)

    def wait(self, ticket: int, timeout_ms: int = -1) -> Result:
        return Result(self._ctx, gpolylla_serve_wait(self.handle, ticket, timeout_ms))

    def stats(self) -> dict:
        return gpolylla_serve_stats(self.handle)

    def reset_stats(self):
        gpolylla_serve_reset_stats(self.handle)

    def stop(self):
        if self.handle:
            gpolylla_serve_stop(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.stop()


class Context:
    def __init__(self, device: int = 0, pool_bytes: int = 0, stream=None, profile: bool = False,
                 block: int = 0, items: int = 0):
        opts = gp_ctx_opts(pool_bytes, int(stream) if stream else None, int(profile), block, items)
        self.handle = gpolylla_ctx_create(device, opts)
        self.device = device

    def build_halfedges(self, xy, tri, flags: int = 0) -> Mesh:
        return Mesh(self, gpolylla_build_halfedges(self.handle, xy, tri, flags, self.device))

    def mesh(self, mesh: Mesh, flags: int = 0) -> Result:
        return Result(self, gpolylla_mesh(self.handle, mesh.handle, flags))

    def mesh_batch(self, meshes, flags: int = 0) -> list:
        hs = gpolylla_mesh_batch(self.handle, [m.handle for m in meshes], flags)
        return [Result(self, h) for h in hs]

    def sync(self):
        gpolylla_ctx_sync(self.handle)

    def kernel_ms(self) -> dict:
        return gpolylla_ctx_kernel_ms(self.handle)

    def kernel_reset(self):
        gpolylla_ctx_kernel_reset(self.handle)

    def set_debug(self, on: bool = True):
        _check(_load().gpolylla_ctx_set_debug(self.handle, int(on)), "gpolylla_ctx_set_debug")

    def set_launch(self, spec: str):
        gpolylla_ctx_set_launch(self.handle, spec)

    def launch(self) -> str:
        return gpolylla_ctx_get_launch(self.handle)

    def pool_bytes(self):
        return gpolylla_ctx_pool_bytes(self.handle)

    def close(self):
        if self.handle:
            gpolylla_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
