"""The compact half-edge encoding (GP_COMPACT): a mesh built compactly gives
the same outputs as the oracle, element by element, including its decoded
corners and twins; meshes whose offsets do not fit 16 bits (scrambled
numberings) go through the escape table; compact and int32 meshes mix in
one batch; the full-size 33.5M-triangle grid meshes identically in both
encodings and holds fewer bytes."""
import sys

import numpy as np
import pytest

import oracle
import paper_2403_14723_amd as gp
from paper_2403_14723_amd import workloads as W
from tests.test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu
KEYS = ("next", "prev", "seeds", "loop_off", "loop_he")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gp.Context(0)
    yield c
    c.close()


def run_compact(ctx, m):
    say(f"[gpu] compact {m.name}: nv={m.nv} nt={m.nt}")
    h = ctx.build_halfedges(m.xy, m.tri, gp.GP_COMPACT)
    org, twin, nflip = h.copy()
    nbytes, nesc = h.nbytes()
    r = ctx.mesh(h)
    g = r.copy()
    r.free()
    h.free()
    g.update(org=org, twin=twin, nflipped=nflip)
    return g, nbytes, nesc


CASES = [W.jittered_grid(40, seed=1001), W.jittered_grid(150, seed=1002, warp=True),
         W.random_delaunay(20000, 1003), W.scrambled(W.random_delaunay(20000, 1004), 5),
         W.scrambled(W.jittered_grid(300, seed=1005), 6), W.flat_strip(800)]


@pytest.mark.parametrize("mesh", CASES, ids=[m.name for m in CASES])
def test_compact_matches_oracle(ctx, mesh):
    g, nbytes, nesc = run_compact(ctx, mesh)
    assert_parity(g, oracle.polylla(mesh.xy, mesh.tri), "compact:" + mesh.name)
    if mesh.name.startswith("scr"):
        assert nesc > 0   # a scrambled numbering cannot fit every offset in 16 bits


def test_compact_delaunay_large_qhull_order(ctx):
    """400k random points in the generator's Qhull order: far neighbours, so
    many escapes, and thousands of barrier tips."""
    m = W.random_delaunay(400000, 1006)
    g, nbytes, nesc = run_compact(ctx, m)
    o = oracle.polylla(m.xy, m.tri)
    assert_parity(g, o, "compact:" + m.name)
    assert o.stats["ntips"] > 1000


def test_compact_and_int32_mix_in_one_batch(ctx):
    meshes = [W.jittered_grid(s, seed=1010 + k, warp=(k % 2 == 0)) for k, s in enumerate([16, 33, 5, 64])]
    meshes.append(W.scrambled(W.random_delaunay(3000, 1015), 7))
    hs = [ctx.build_halfedges(m.xy, m.tri, gp.GP_COMPACT if k % 2 else 0) for k, m in enumerate(meshes)]
    say(f"[gpu] compact/int32 batch of {len(hs)}")
    rs = ctx.mesh_batch(hs)
    for m, h, r in zip(meshes, hs, rs):
        g = r.copy()
        org, twin, nflip = h.copy()
        g.update(org=org, twin=twin, nflipped=nflip)
        assert_parity(g, oracle.polylla(m.xy, m.tri), "batch:" + m.name)
        r.free()
        h.free()


def test_compact_full_size_grid(ctx):
    """The 33.5M-triangle warped grid: compact and int32 meshes give
    identical outputs (the int32 path is compared with the oracle at this
    size in the parity suite) and the compact one holds fewer bytes."""
    m = W.plain_large_warped()
    say("[gpu] compact full-size grid")
    outs, sizes = [], []
    for flags in (0, gp.GP_COMPACT):
        h = ctx.build_halfedges(m.xy, m.tri, flags)
        sizes.append(h.nbytes())
        r = ctx.mesh(h)
        outs.append(r.copy())
        r.free()
        if flags:
            org, twin, _ = h.copy()
        h.free()
    for k in KEYS:
        assert np.array_equal(outs[0][k], outs[1][k]), k
    assert sizes[1][0] < 0.8 * sizes[0][0], sizes
    assert sizes[1][1] == 0   # row-ordered: every offset fits
    o_org, o_twin, _ = oracle.build(m.xy, m.tri)
    assert np.array_equal(org, o_org) and np.array_equal(twin, o_twin)
