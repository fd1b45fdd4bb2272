"""The launch-shape autotuner: it returns a valid spec, caches it per workload
signature, and the batch meshed under the tuned shapes equals the oracle."""
import numpy as np
import pytest

import oracle
import paper_2403_14723_amd as gp
from paper_2403_14723_amd import autotune
from paper_2403_14723_amd import workloads as W
from tests.test_gpu_parity import assert_parity, say

pytestmark = pytest.mark.gpu


def test_tune_cache_and_parity(tmp_path):
    meshes = [W.jittered_grid(s, seed=500 + k, warp=(k % 2 == 0)) for k, s in enumerate([40, 7, 90, 23])]
    meshes.append(W.random_delaunay(5000, 501))
    cache = str(tmp_path / "tune.json")
    say("[gpu] autotune search")
    first = autotune.tune(meshes, reps=1, cache=cache)
    assert not first["cached"]
    assert set(autotune.GROUPS) <= set(first["ms"])
    second = autotune.tune(meshes, reps=1, cache=cache)
    assert second["cached"] and second["spec"] == first["spec"]
    with gp.Context(0) as c:
        c.set_launch(first["spec"])
        assert c.launch().startswith(first["spec"] + ",small=")
        hs = [c.build_halfedges(m.xy, m.tri) for m in meshes]
        rs = c.mesh_batch(hs, gp.GP_GRAPH)
        for m, h, r in zip(meshes, hs, rs):
            got = r.copy()
            org, twin, nflip = h.copy()
            got.update(org=org, twin=twin, nflipped=nflip)
            assert_parity(got, oracle.polylla(m.xy, m.tri), "tuned:" + m.name)
            r.free()
        for h in hs:
            h.free()
