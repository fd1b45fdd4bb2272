"""GPU parity: the HIP path, called through the C ABI, against the oracle.

Every output array is compared element by element (integer work: bit-exact)
on the same seeded inputs: hand-made fixtures, small jittered / warped grids,
Delaunay meshes of random points (many barrier tips), the paper's clockwise
grid, the 32x32 and 1024x1024 workloads, and the 4096x4096 warped workload at
full size in the launch configuration the benchmark uses.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2403_14723_amd as gp
from paper_2403_14723_amd import workloads as W
from tests import polycheck as pc

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gp.Context(0)
    yield c
    c.close()


def run_gpu(ctx, xy, tri, name=""):
    say(f"[gpu] {name}: nv={len(xy)} nt={len(tri)}")
    m = ctx.build_halfedges(xy, tri)
    org, twin, nflip = m.copy()
    r = ctx.mesh(m)
    out = r.copy()
    r.free()
    m.free()
    out.update(org=org, twin=twin, nflipped=nflip)
    return out


def assert_parity(g, o, name=""):
    for key, a, b in (("org", g["org"], o.org), ("twin", g["twin"], o.twin), ("next", g["next"], o.next),
                      ("prev", g["prev"], o.prev), ("seeds", g["seeds"], o.seeds),
                      ("loop_off", g["loop_off"], o.loop_off), ("loop_he", g["loop_he"], o.loop_he)):
        assert a.shape == b.shape, f"{name}: {key} shape {a.shape} vs {b.shape}"
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{name}: {key} differs at {len(bad)} positions, first {bad[:5]}: "
                                 f"gpu {a[bad[:5]]} oracle {b[bad[:5]]}")
    info = g["info"]
    for k in ("npoly", "nloop_he", "nterminal", "ntips", "nmiddle", "nties"):
        assert info[k] == o.stats[k], f"{name}: {k} gpu {info[k]} oracle {o.stats[k]}"
    assert g["nflipped"] == o.stats["nflipped"]


def check_case(ctx, xy, tri, name):
    o = oracle.polylla(xy, tri)
    g = run_gpu(ctx, xy, tri, name)
    assert_parity(g, o, name)
    return g, o


FIXTURES = ["p1_two_triangles_square.txt", "p2_one_triangle.txt", "p3_fan_degree8.txt",
            "p4_fan_degree7.txt", "p_tie_break.txt"]


@pytest.mark.parametrize("name", FIXTURES)
def test_fixtures(ctx, name):
    fx = pc.load_fixture(name)
    check_case(ctx, fx["xy"], fx["tri"], name)


def _small_cases():
    out = []
    for n in (1, 2, 3, 7, 16, 33, 64):
        for seed in range(3):
            out.append(W.jittered_grid(n, seed=seed))
    for n, seed in ((24, 100), (40, 101), (96, 102)):
        out.append(W.jittered_grid(n, seed=seed, warp=True))
    for n in (5, 12):
        out.append(W.jittered_grid(n, seed=7, jitter=0.0))
    for npts, seed in ((10, 1), (300, 2), (5000, 3), (60000, 4)):
        out.append(W.random_delaunay(npts, seed))
    out.append(W.random_delaunay(60000, 9, order="morton"))   # spatially ordered numbering
    return out


SMALL = _small_cases()


@pytest.mark.parametrize("mesh", SMALL, ids=[m.name for m in SMALL])
def test_small(ctx, mesh):
    check_case(ctx, mesh.xy, mesh.tri, mesh.name)


def test_paper_grid_clockwise(ctx):
    xy, tri = pc.paper_grid(2500)
    g, o = check_case(ctx, xy, tri, "paper_grid_2500")
    assert g["nflipped"] == len(tri)


def test_plain_small_workload(ctx):
    m = W.plain_small()
    g, o = check_case(ctx, m.xy, m.tri, m.name)
    pc.check_output(m.xy, g["org"], g["twin"], g["next"], g["prev"], g["seeds"], g["loop_off"],
                    g["loop_he"])


def test_plain_scale_workload(ctx):
    m = W.plain_scale()
    check_case(ctx, m.xy, m.tri, m.name)


def test_delaunay_large(ctx):
    m = W.random_delaunay(400000, 11)
    g, o = check_case(ctx, m.xy, m.tri, m.name)
    assert o.stats["ntips"] > 1000


def test_plain_large_warped_full(ctx):
    """The 33.5M-triangle workload at full size, default launch configuration
    (the one the benchmark times), every output element compared; then the
    benchmark's band form of it (band 3 of 8 row bands, two halo rows) against
    the oracle, and its band proper against the whole mesh."""
    m = W.plain_large_warped()
    g, o = check_case(ctx, m.xy, m.tri, m.name)
    assert o.stats["ntips"] > 0
    del o
    n, nb, b = 4096, 8, 3
    rows = n // nb
    bm = W.grid_band(m, n, b, nb)
    gb, _ = check_case(ctx, bm.xy, bm.tri, bm.name)
    off = 6 * n * (b * rows - 2)
    lo, hi = 6 * n * b * rows - off, 6 * n * (b + 1) * rows - off
    for key in ("next", "prev"):
        got = gb[key][lo:hi]
        np.testing.assert_array_equal(np.where(got >= 0, got + off, -1), g[key][lo + off:hi + off])


def test_delaunay_1m_workload(ctx):
    """The benchmark's general-position workload at full size (1M random
    points, Z-order numbering, 1,979,675 triangles), every element compared."""
    m = W.delaunay_1m()
    assert m.nt == 1979675
    g, o = check_case(ctx, m.xy, m.tri, m.name)
    assert o.stats["ntips"] > 10000


def test_batch_equals_plain(ctx):
    meshes = [W.jittered_grid(s, seed=900 + k, warp=(k % 3 == 0)) for k, s in
              enumerate([16, 1, 40, 23, 64, 5, 100, 37])] + [W.random_delaunay(3000, 77)]
    hs = [ctx.build_halfedges(m.xy, m.tri) for m in meshes]
    say(f"[gpu] batch of {len(hs)}")
    rs = ctx.mesh_batch(hs)
    for m, h, r in zip(meshes, hs, rs):
        got = r.copy()
        o = oracle.polylla(m.xy, m.tri)
        org, twin, nflip = h.copy()
        got.update(org=org, twin=twin, nflipped=nflip)
        assert_parity(got, o, "batch:" + m.name)
        r.free()
    # a mesh may appear twice in one batch
    rs = ctx.mesh_batch([hs[2], hs[2]])
    a, b = rs[0].copy(), rs[1].copy()
    for k in ("next", "prev", "seeds", "loop_off", "loop_he"):
        assert np.array_equal(a[k], b[k])
    for r in rs:
        r.free()
    for h in hs:
        h.free()


@pytest.mark.parametrize("block,items", [(64, 1), (128, 2), (512, 8), (1024, 4)])
def test_launch_shapes_do_not_change_results(block, items):
    m = W.jittered_grid(150, seed=31, warp=True)
    o = oracle.polylla(m.xy, m.tri)
    with gp.Context(0, block=block, items=items) as c:
        g = run_gpu(c, m.xy, m.tri, f"{m.name} block={block} items={items}")
    assert_parity(g, o, f"block={block},items={items}")


def test_repeat_and_async_identical(ctx):
    m = W.random_delaunay(20000, 5)
    h = ctx.build_halfedges(m.xy, m.tri)
    say("[gpu] repeat/async")
    rs = [ctx.mesh(h, gp.GP_ASYNC) for _ in range(4)]
    outs = [r.copy() for r in rs]
    for r in rs:
        r.free()
    for k in ("next", "prev", "seeds", "loop_off", "loop_he"):
        for o in outs[1:]:
            assert np.array_equal(outs[0][k], o[k])
    h.free()


def test_device_inputs_from_torch(ctx):
    import torch
    m = W.jittered_grid(50, seed=3)
    xy = torch.from_numpy(m.xy).cuda()
    tri = torch.from_numpy(m.tri).cuda()
    torch.cuda.synchronize()
    say("[gpu] torch device inputs")
    h = ctx.build_halfedges(xy, tri)
    r = ctx.mesh(h)
    g = r.copy()
    org, twin, nflip = h.copy()
    g.update(org=org, twin=twin, nflipped=nflip)
    assert_parity(g, oracle.polylla(m.xy, m.tri), "torch-input")
    r.free()
    h.free()


def test_empty_mesh(ctx):
    say("[gpu] empty")
    h = ctx.build_halfedges(np.zeros((0, 2), np.int32), np.zeros((0, 3), np.int32))
    r = ctx.mesh(h)
    g = r.copy()
    assert g["info"]["npoly"] == 0 and list(g["loop_off"]) == [0]
    r.free()
    h.free()


@pytest.mark.parametrize("case", ["nonmanifold", "duplicate", "zero_area", "index", "coord"])
def test_build_errors_match_oracle(ctx, case):
    xy, tri = {
        "nonmanifold": ([[0, 10], [10, 10], [5, 15], [5, 5], [5, 19]], [[0, 1, 2], [1, 0, 3], [0, 1, 4]]),
        "duplicate": ([[0, 0], [10, 0], [5, 5]], [[0, 1, 2], [0, 1, 2]]),
        "zero_area": ([[0, 0], [1, 1], [2, 2]], [[0, 1, 2]]),
        "index": ([[0, 0], [1, 0], [0, 1]], [[0, 1, 3]]),
        "coord": ([[0, 0], [(1 << 30) + 1, 0], [0, 1]], [[0, 1, 2]]),
    }[case]
    xy, tri = np.array(xy, np.int32), np.array(tri, np.int32)
    with pytest.raises(oracle.OracleError) as eo:
        oracle.polylla(xy, tri)
    say(f"[gpu] build error {case}")
    with pytest.raises(gp.GPolyllaError) as eg:
        ctx.build_halfedges(xy, tri)
    assert eg.value.code == eo.value.code


def test_graph_replays_match_eager(ctx):
    """The captured chain, replayed several times with eager runs and syncs in
    between, gives the eager result every time (one mesh and a batch)."""
    meshes = [W.jittered_grid(40, seed=71, warp=True), W.random_delaunay(4000, 72),
              W.jittered_grid(9, seed=73)]
    hs = [ctx.build_halfedges(m.xy, m.tri) for m in meshes]
    eager = [ctx.mesh(h).copy() for h in hs]
    keys = ("next", "prev", "seeds", "loop_off", "loop_he")
    for rep in range(4):
        say(f"[gpu] graph replay {rep}")
        r = ctx.mesh(hs[0], gp.GP_GRAPH)
        got = r.copy()
        r.free()
        for k in keys:
            assert np.array_equal(got[k], eager[0][k]), (rep, k)
        rs = ctx.mesh_batch(hs, gp.GP_GRAPH)
        for i, rr in enumerate(rs):
            got = rr.copy()
            for k in keys:
                assert np.array_equal(got[k], eager[i][k]), (rep, i, k)
            rr.free()
        # eager work and a sync between replays
        e = ctx.mesh(hs[1])
        e.free()
        ctx.sync()
    for h in hs:
        h.free()


def test_launch_spec_roundtrip_and_errors():
    with gp.Context(0) as c:
        c.set_launch("label=512x2,relink=128x4,compact=256x8,persist=256x512,small=1000")
        assert c.launch() == "label=512x2,relink=128x4,compact=256x8,persist=256x512,small=1000"
        before = c.launch()
        for bad in ("label=100x2", "relink=256x3", "nope=256x2", "label=256", "label=x2", "label=256x2,,x",
                    "compact=2048x1", "persist=256x0", "label=256x2;relink=256x2", "small=4097", "small=",
                    "small=-1", "small=1x2"):
            with pytest.raises(gp.GPolyllaError) as e:
                c.set_launch(bad)
            assert e.value.code == gp.GP_EINVAL, bad
            assert c.launch() == before, bad
        # tiles beyond the LDS staging are clamped by halving the items
        c.set_launch("relink=1024x8,label=1024x8,compact=1024x8")
        assert c.launch().startswith("label=1024x4,relink=1024x1,compact=1024x2")


@pytest.mark.parametrize("spec", ["label=64x1,relink=64x1,compact=64x1,persist=64x1",
                                  "label=1024x4,relink=128x8,compact=128x8,persist=1024x4096",
                                  # compaction tiles smaller than relink's: 8 per relink tile, and
                                  # 384-triangle relink tiles straddling 256-triangle ones
                                  "relink=256x4,compact=64x2",
                                  "label=192x1,relink=192x2,compact=256x1,persist=192x100"])
def test_launch_specs_do_not_change_results(spec):
    m = W.random_delaunay(20000, 41)
    o = oracle.polylla(m.xy, m.tri)
    with gp.Context(0) as c:
        c.set_launch(spec)
        g = run_gpu(c, m.xy, m.tri, f"{m.name} {spec}")
    assert_parity(g, o, spec)


def _wheel(n):
    """n triangles around one centre, radii growing around the rim: every spoke
    but the first is the longest edge of a triangle, so the centre is a
    barrier tip of degree n (fix-up turns around a vertex of any degree)."""
    import math
    c = 1 << 19
    pts = [[c, c]] + [[int(c + 200000 * (1 + 0.3 * k / n) * math.cos(2 * math.pi * k / n)),
                       int(c + 200000 * (1 + 0.3 * k / n) * math.sin(2 * math.pi * k / n))] for k in range(n)]
    tri = [[0, 1 + k, 1 + (k + 1) % n] for k in range(n)]
    return np.array(pts, np.int32), np.array(tri, np.int32)


@pytest.mark.parametrize("n", [12, 20, 40, 64])
def test_wheel_tip_of_high_degree(ctx, n):
    xy, tri = _wheel(n)
    g, o = check_case(ctx, xy, tri, f"wheel{n}")
    assert o.stats["ntips"] == 1


def test_grid_bands(ctx):
    """One device's share of a row-band split with two halo rows: every band
    meshes like any mesh, and the half-edges of its band proper get the whole
    grid's next'/prev' (shifted by the cut)."""
    n, nb = 256, 8
    m = W.jittered_grid(n, seed=41, warp=True)
    whole, _ = check_case(ctx, m.xy, m.tri, m.name)
    rows = n // nb
    for b in range(nb):
        bm = W.grid_band(m, n, b, nb)
        g, _ = check_case(ctx, bm.xy, bm.tri, bm.name)
        off = 6 * n * max(0, b * rows - 2)
        lo, hi = 6 * n * b * rows - off, 6 * n * (b + 1) * rows - off
        for key in ("next", "prev"):
            got = g[key][lo:hi]
            np.testing.assert_array_equal(np.where(got >= 0, got + off, -1), whole[key][lo + off:hi + off])


def _tall_strip(n):
    """flat_strip stretched 8x upwards: in every triangle the two slanted
    sides are the longest edges, and exactly equal when the base width
    2^20 // n is even, so that every label is a tie."""
    assert ((1 << 20) // n) % 2 == 0
    m = W.flat_strip(n)
    xy = m.xy.copy()
    xy[:, 1] *= 8
    return W.Mesh(xy, m.tri, f"tall_strip{n}")


SCRAMBLED = [W.scrambled(W.jittered_grid(96, seed=5, warp=True), 1),
             W.scrambled(_tall_strip(1000), 2),
             W.scrambled(W.random_delaunay(20000, 8), 3),
             W.scrambled(W.flat_strip(1500), 4)]


@pytest.mark.parametrize("mesh", SCRAMBLED, ids=[m.name for m in SCRAMBLED])
def test_scrambled_numbering(ctx, mesh):
    """Random vertex and triangle order, rotated corners, mixed orientation:
    most neighbours lie in other tiles, and ties fall among scattered ids."""
    g, o = check_case(ctx, mesh.xy, mesh.tri, mesh.name)
    assert g["nflipped"] > 0
    if mesh.name.startswith("tall_strip"):
        assert o.stats["nties"] == mesh.nt


@pytest.mark.parametrize("n", [600, 5000])
def test_flat_strip_every_triangle_a_polygon(ctx, n):
    """Three loop half-edges per triangle, more than a compaction tile keeps
    in LDS: those tiles write their loops straight to global memory."""
    m = W.flat_strip(n)
    g, o = check_case(ctx, m.xy, m.tri, m.name)
    assert o.stats["npoly"] == m.nt


@pytest.mark.parametrize("case", ["hole", "two"])
def test_hole_and_two_components(ctx, case):
    """An inner boundary (a grid with a hole; its vertices unused) and two
    disjoint components, against the oracle and the invariants."""
    xy, tri, chi = pc.grid_with_hole(96, 17, 30) if case == "hole" else pc.two_grids(70, 45, 18)
    g, o = check_case(ctx, xy, tri, case)
    pc.check_output(xy, g["org"], g["twin"], g["next"], g["prev"], g["seeds"], g["loop_off"], g["loop_he"],
                    chi=chi)


def test_loops_longer_than_the_length_code(ctx):
    """One polygon per rising strip, loops of 62 to 66, 127, 1,001 and 4,001
    half-edges (5,433 triangles, so the tiled chain runs): the walk, the
    lengths of loops longer than a loop byte holds, and the emitted loops,
    against the oracle."""
    cases = [(30, True), (31, False), (31, True), (32, False), (32, True), (63, False), (500, False), (2000, False)]
    xy, tri, chi, lens = pc.rising_strips(cases)
    assert len(tri) > 4096
    g, o = check_case(ctx, xy, tri, "rising_strips")
    np.testing.assert_array_equal(np.diff(g["loop_off"]), lens)
    pc.check_output(xy, g["org"], g["twin"], g["next"], g["prev"], g["seeds"], g["loop_off"], g["loop_he"],
                    chi=chi)


def test_pool_exhaustion_is_an_error_and_the_context_recovers():
    """A context whose device pool is capped refuses a mesh that does not fit
    with GP_ENOMEM (nothing is launched for it) and still meshes one that
    does."""
    big, small = W.jittered_grid(800, seed=3), W.jittered_grid(8, seed=3)
    with gp.Context(0, pool_bytes=16 << 20) as c:
        say("[gpu] capped pool: build that does not fit")
        with pytest.raises(gp.GPolyllaError) as e:
            c.build_halfedges(big.xy, big.tri)
        assert e.value.code == gp.GP_ENOMEM
        g = run_gpu(c, small.xy, small.tri, "after ENOMEM")
    assert_parity(g, oracle.polylla(small.xy, small.tri), "after ENOMEM")
