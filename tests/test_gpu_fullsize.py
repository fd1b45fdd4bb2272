"""Parity at the full sizes of the batched and served workloads, in the launch
configurations the benchmark times.

* Batched: the 512 meshes of the batched workload (about 35.6M triangles) run
  as one captured batch, with the default launch shapes and with the shapes
  the autotuner picks; every output element of every mesh is compared with
  the oracle.
* Served: all 2,000 requests of the served workload go through a server set
  up like the benchmark's (3 lanes, batches of up to 32).  Requests that carry
  the same mesh must give identical results; a fixed sample of the distinct
  meshes (the largest among them) is compared element by element with the
  oracle, and every result's counts with those of the mesh's first result.
"""
import hashlib
import sys

import numpy as np
import pytest

import oracle
import paper_2403_14723_amd as gp
from paper_2403_14723_amd import autotune
from paper_2403_14723_amd import workloads as W
from tests.test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu
KEYS = ("next", "prev", "seeds", "loop_off", "loop_he")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _digest(res: dict) -> str:
    h = hashlib.sha256()
    for k in KEYS:
        h.update(np.ascontiguousarray(res[k]).tobytes())
        h.update(b"|")
    return h.hexdigest()


def _assert_outputs(g, o, name):
    """The outputs a served result carries (no org/twin) against the oracle."""
    for k in KEYS:
        a, b = g[k], getattr(o, k)
        assert a.shape == b.shape, f"{name}: {k} shape {a.shape} vs {b.shape}"
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{name}: {k} differs at {len(bad)} positions, first {bad[:5]}")
    for k in ("npoly", "nloop_he", "nterminal", "ntips", "nmiddle", "nties"):
        assert g["info"][k] == o.stats[k], f"{name}: {k} gpu {g['info'][k]} oracle {o.stats[k]}"


def test_batched_workload_full(tmp_path):
    meshes = W.batch_meshes(512, seed=3)
    say(f"[gpu] batched: {len(meshes)} meshes, {sum(m.nt for m in meshes)} triangles; autotune")
    tuned = autotune.tune(meshes, cache=str(tmp_path / "tune.json"))
    with gp.Context(0) as c:
        specs = [c.launch(), tuned["spec"]]
        hs = [c.build_halfedges(m.xy, m.tri) for m in meshes]
        digests = None
        for spec in specs:
            say(f"[gpu] batched run with {spec}")
            c.set_launch(spec)
            rs = c.mesh_batch(hs, gp.GP_GRAPH)
            got = []
            for r in rs:
                got.append(_digest(r.copy()) if digests is not None else r.copy())
                r.free()
            if digests is None:
                digests = []
                for m, h, g in zip(meshes, hs, got):
                    org, twin, nflip = h.copy()
                    g.update(org=org, twin=twin, nflipped=nflip)
                    assert_parity(g, oracle.polylla(m.xy, m.tri), "batch:" + m.name)
                    digests.append(_digest(g))
                got = None
            else:
                assert got == digests, "tuned launch shapes changed a result"
        for h in hs:
            h.free()


def test_served_workload_full_sampled():
    reqs = W.served_requests(2000)
    distinct = list({id(m): m for m in reqs}.values())
    by_size = sorted(distinct, key=lambda m: m.nt)
    # the oracle sample: the largest distinct mesh and seven spread over the sizes
    sample = {id(by_size[int(round(q * (len(by_size) - 1)))]) for q in np.linspace(0, 1, 8)}
    say(f"[gpu] served: {len(reqs)} requests, {len(distinct)} distinct meshes, "
        f"{sum(m.nt for m in reqs)} triangles")
    first: dict = {}
    checked = set()
    window = 64
    with gp.Context(0) as ctx, gp.Server(ctx, pool_bytes=48 << 30, max_batch=32, n_lanes=3) as srv:
        for w0 in range(0, len(reqs), window):
            part = reqs[w0:w0 + window]
            tickets = [srv.submit(m.xy, m.tri) for m in part]
            for k, (m, t) in enumerate(zip(part, tickets)):
                r = srv.wait(t, 120000)
                info = r.info()
                if id(m) not in first or (w0 + k) % 8 == 0:
                    g = r.copy()
                    d = _digest(g)
                    if id(m) not in first:
                        first[id(m)] = (d, info)
                        if id(m) in sample:
                            _assert_outputs(g, oracle.polylla(m.xy, m.tri), "served:" + m.name)
                            checked.add(id(m))
                    else:
                        assert d == first[id(m)][0], ("request", w0 + k, m.name)
                    del g
                assert info == first[id(m)][1], ("request", w0 + k, m.name)
                r.free()
        st = srv.stats()
    assert st["failed"] == 0 and st["completed"] == len(reqs)
    assert checked == sample and len(first) == len(distinct)
