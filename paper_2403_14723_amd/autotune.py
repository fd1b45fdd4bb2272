"""Launch-shape autotuner for the meshing pipeline.

The launch shapes (threads per block, triangles per thread, persistent grid
size) never change a result; they only move time between latency and
occupancy, and the best ones depend on the workload's mesh sizes.  The search
is coordinate-wise: for every kernel group in turn, each candidate shape is
timed on the caller's meshes and the fastest one is kept.  The time is that
of the whole chain (per-kernel HIP event times from a profiling context,
summed, averaged over several batched runs): one kernel's shape also moves
work in others (the compaction tile sets the tile scan's length and how the
relink tiles feed it).  The starting shapes stay unless the search beats
them.

Results are cached in a JSON file keyed by the device and a signature of the
workload (mesh count and total triangles, rounded to a power of two), so a
second call with a like workload costs nothing.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import GP_ASYNC, Context

# kernel group -> (the kernels it shapes, candidate (B, I) shapes)
GROUPS = {
    "label": (("k_label",), [(b, i) for b in (128, 256, 512, 1024) for i in (1, 2, 4, 8) if b * i <= 4096]),
    "relink": (("k_relink",), [(b, i) for b in (64, 128, 256, 512, 1024) for i in (1, 2, 4, 8) if b * i <= 1024]),
    "compact": (("k_compact",), [(b, i) for b in (128, 256, 512, 1024) for i in (1, 2, 4, 8) if b * i <= 2048]),
    # list-driven kernels: 256 threads per block, N blocks
    "persist": (("k_repair", "k_fixup", "k_walk", "k_emit"), [(256, n) for n in (256, 512, 1024, 2048, 4096)]),
}


def default_cache_path() -> str:
    root = os.environ.get("GPOLYLLA_TUNE_CACHE")
    if root:
        return root
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "gpolylla", "autotune.json")


def workload_key(device: int, nts) -> str:
    import torch
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", props.name)
    total = max(1, int(sum(nts)))
    return f"{arch}|meshes={len(nts)}|T~2^{round(math.log2(total))}"


def _spec(shapes: dict) -> str:
    return ",".join(f"{k}={b}x{i}" for k, (b, i) in shapes.items())


def _parse(spec: str) -> dict:
    """The "kernel=BxI" entries of a launch spec (other entries, such as
    the small-mesh limit, are not tuned and are left as they are)."""
    out = {}
    for item in spec.split(","):
        k, v = item.split("=")
        if "x" not in v:
            continue
        b, i = v.split("x")
        out[k] = (int(b), int(i))
    return out


def _time_chain(ctx: Context, handles, reps: int) -> float:
    for r in ctx.mesh_batch(handles, GP_ASYNC):   # warm-up (first-use allocations)
        r.free()
    ctx.sync()
    ctx.kernel_reset()
    for _ in range(reps):
        for r in ctx.mesh_batch(handles, GP_ASYNC):
            r.free()
    ctx.sync()
    return sum(avg for avg, _ in ctx.kernel_ms().values())


def tune(meshes, device: int = 0, reps: int = 3, cache: str | None = None, force: bool = False,
         log=None) -> dict:
    """Picks launch shapes for `meshes` (objects with host arrays .xy, .tri).

    Returns {"spec": str, "key": str, "ms": {group: best ms}, "seconds": float,
    "cached": bool}; pass "spec" to Context.set_launch.
    """
    t0 = time.perf_counter()
    nts = [int(m.tri.shape[0]) for m in meshes]
    key = workload_key(device, nts)
    path = cache or default_cache_path()
    table = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if not force and key in table:
        hit = dict(table[key])
        hit.update(cached=True, seconds=time.perf_counter() - t0)
        return hit

    with Context(device, profile=True) as ctx:
        start = _parse(ctx.launch())
        shapes = dict(start)
        handles = [ctx.build_halfedges(m.xy, m.tri) for m in meshes]
        best_ms = {}
        try:
            ctx.set_launch(_spec(start))
            start_ms = _time_chain(ctx, handles, reps)
            current = start_ms
            for group, (_kernels, cands) in GROUPS.items():
                best = (current, shapes[group])
                for cand in cands:
                    if cand == shapes[group]:
                        continue
                    trial = dict(shapes)
                    trial[group] = cand
                    ctx.set_launch(_spec(trial))
                    if _parse(ctx.launch())[group] != cand:
                        continue   # clamped to a shape already tried
                    ms = _time_chain(ctx, handles, reps)
                    if log:
                        log(f"[tune] {group}={cand[0]}x{cand[1]}: {ms:.4f} ms")
                    if ms < best[0]:
                        best = (ms, cand)
                shapes[group] = best[1]
                best_ms[group] = round(best[0], 5)
                current = best[0]
            # confirm against the starting shapes, both timed again
            ctx.set_launch(_spec(shapes))
            tuned_ms = _time_chain(ctx, handles, 2 * reps)
            ctx.set_launch(_spec(start))
            again_ms = _time_chain(ctx, handles, 2 * reps)
            if tuned_ms >= again_ms:
                shapes = start
            best_ms["chain_start"] = round(again_ms, 5)
            best_ms["chain_tuned"] = round(tuned_ms, 5)
        finally:
            for h in handles:
                h.free()
    entry = {"spec": _spec(shapes), "key": key, "ms": best_ms}
    table[key] = entry
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass   # an unwritable cache only costs the next call a search
    out = dict(entry)
    out.update(cached=False, seconds=time.perf_counter() - t0)
    return out
