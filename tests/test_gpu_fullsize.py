"""Parity at the full sizes of the batched and served workloads, in the launch
configurations the benchmark times.

* Batched: the 512 meshes of the batched workload (about 35.6M triangles) run
  as one captured batch, with the default launch shapes and with the shapes
  the autotuner picks; every output element of every mesh is compared with
  the oracle.
* Served: all 2,000 requests of the served workload go through a server set
  up like the benchmark's (3 lanes, batches of up to 32).  The first result
  of each of the 192 distinct meshes is compared with the oracle's outputs
  (a digest of every output element) and counts; requests that carry the
  same mesh must give identical counts, and every eighth one identical
  outputs.
"""
import hashlib
import sys
from concurrent.futures import ThreadPoolExecutor

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


def _oracle_digest(m):
    o = oracle.polylla(m.xy, m.tri)
    stats = {k: o.stats[k] for k in ("npoly", "nloop_he", "nterminal", "ntips", "nmiddle", "nties")}
    return _digest({k: getattr(o, k) for k in KEYS}), stats


def test_served_workload_full():
    reqs = W.served_requests(2000)
    distinct = list({id(m): m for m in reqs}.values())
    say(f"[gpu] served: {len(reqs)} requests, {len(distinct)} distinct meshes, "
        f"{sum(m.nt for m in reqs)} triangles")
    # the oracle's outputs of every distinct mesh, computed on host threads
    # while the server runs (the oracle's C core releases the GIL)
    pool = ThreadPoolExecutor(max_workers=8)
    want = {id(m): pool.submit(_oracle_digest, m) for m in distinct}
    first: dict = {}
    window = 64
    with gp.Context(0) as ctx, gp.Server(ctx, pool_bytes=48 << 30, max_batch=32, n_lanes=3) as srv:
        for w0 in range(0, len(reqs), window):
            part = reqs[w0:w0 + window]
            tickets = [srv.submit(m.xy, m.tri) for m in part]
            for k, (m, t) in enumerate(zip(part, tickets)):
                r = srv.wait(t, 120000)
                info = r.info()
                if id(m) not in first or (w0 + k) % 8 == 0:
                    d = _digest(r.copy())
                    if id(m) not in first:
                        first[id(m)] = (d, info)
                    else:
                        assert d == first[id(m)][0], ("request", w0 + k, m.name)
                assert info == first[id(m)][1], ("request", w0 + k, m.name)
                r.free()
        st = srv.stats()
    assert st["failed"] == 0 and st["completed"] == len(reqs)
    assert len(first) == len(distinct)
    say("[gpu] served: comparing every distinct mesh with the oracle")
    bad = []
    for m in distinct:
        d, stats = want[id(m)].result()
        g, info = first[id(m)]
        if d != g or any(info[k] != v for k, v in stats.items()):
            bad.append(m.name)
    pool.shutdown()
    assert not bad, f"{len(bad)} served meshes differ from the oracle: {bad[:8]}"
