"""Renumbering along a Z-order curve inside the build (GP_RENUMBER): the maps
are permutations, and every output equals the oracle's on the input
renumbered by those maps on the host, element by element (so ties fall as the
new numbering breaks them); it combines with the compact encoding and with
device inputs; input errors are reported as without it."""
import sys

import numpy as np
import pytest

import oracle
import paper_2403_14723_amd as gp
from paper_2403_14723_amd import workloads as W
from tests.test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gp.Context(0)
    yield c
    c.close()


def renumbered_input(m, tp, vp):
    assert np.array_equal(np.sort(tp), np.arange(m.nt)) and np.array_equal(np.sort(vp), np.arange(m.nv))
    vinv = np.empty(m.nv, np.int64)
    vinv[vp] = np.arange(m.nv)
    return m.xy[vp], vinv[m.tri[tp]].astype(np.int32)


def run_renumbered(ctx, m, flags=0, xy=None, tri=None):
    say(f"[gpu] renumber {m.name}: nt={m.nt} flags={flags}")
    h = ctx.build_halfedges(m.xy if xy is None else xy, m.tri if tri is None else tri, gp.GP_RENUMBER | flags)
    tp, vp = h.permutation()
    org, twin, nflip = h.copy()
    r = ctx.mesh(h)
    g = r.copy()
    r.free()
    h.free()
    g.update(org=org, twin=twin, nflipped=nflip)
    return g, tp, vp


CASES = [W.scrambled(W.random_delaunay(20000, 1201), 3), W.random_delaunay(30000, 1202),
         W.scrambled(W.jittered_grid(120, seed=1203, warp=True), 4), W.jittered_grid(64, seed=1204),
         W.flat_strip(500)]


@pytest.mark.parametrize("mesh", CASES, ids=[m.name for m in CASES])
def test_renumbered_matches_oracle(ctx, mesh):
    g, tp, vp = run_renumbered(ctx, mesh)
    xy2, tri2 = renumbered_input(mesh, tp, vp)
    assert_parity(g, oracle.polylla(xy2, tri2), "renumbered:" + mesh.name)


def test_renumbered_compact_and_device_inputs(ctx):
    import torch
    m = W.scrambled(W.random_delaunay(15000, 1205), 5)
    dev = torch.device("cuda", 0)
    xy_d = torch.from_numpy(np.ascontiguousarray(m.xy)).to(dev)
    tri_d = torch.from_numpy(np.ascontiguousarray(m.tri)).to(dev)
    torch.cuda.synchronize()
    g, tp, vp = run_renumbered(ctx, m, gp.GP_COMPACT | gp.GP_IN_DEVICE, xy_d, tri_d)
    xy2, tri2 = renumbered_input(m, tp, vp)
    assert_parity(g, oracle.polylla(xy2, tri2), "renumbered compact:" + m.name)


def test_renumbered_delaunay_1m_qhull_order(ctx):
    """The general-position workload at full size in the triangulator's own
    order, renumbered by the build."""
    m = W.random_delaunay(1_000_000, 21, order="qhull")
    g, tp, vp = run_renumbered(ctx, m)
    xy2, tri2 = renumbered_input(m, tp, vp)
    o = oracle.polylla(xy2, tri2)
    assert_parity(g, o, "renumbered:" + m.name)
    assert o.stats["ntips"] > 10000


@pytest.mark.parametrize("case", ["index", "zero_area"])
def test_renumbered_input_errors(ctx, case):
    m = W.jittered_grid(10, seed=1206)
    tri = m.tri.copy()
    if case == "index":
        tri[7, 1] = m.nv + 5
    else:
        tri[7, 2] = tri[7, 1]
    want = None
    try:
        oracle.polylla(m.xy, tri)
    except oracle.OracleError as e:
        want = e.code
    assert want is not None
    for flags in (0, gp.GP_RENUMBER):
        with pytest.raises(gp.GPolyllaError) as e:
            ctx.build_halfedges(m.xy, tri, flags)
        assert e.value.code == want, (case, flags)
    with pytest.raises(gp.GPolyllaError):
        h = ctx.build_halfedges(m.xy, m.tri)
        try:
            h.permutation()   # not renumbered
        finally:
            h.free()
