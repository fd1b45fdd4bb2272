"""The one-workgroup form of small meshes (k_small): every mesh of at most
4096 triangles whose arrays fit a workgroup's LDS runs as one launch.  Its
outputs equal the oracle's and the tiled chain's (the same context with
small=0) element by element, for single meshes, batches of small meshes,
captured graphs and compact meshes (integer outputs: tolerance zero)."""
import sys

import numpy as np
import pytest

import oracle
import paper_2403_14723_amd as gp
from paper_2403_14723_amd import workloads as W
from tests import polycheck as pc
from tests.test_gpu_parity import _tall_strip, _wheel, assert_parity

pytestmark = pytest.mark.gpu
KEYS = ("next", "prev", "seeds", "loop_off", "loop_he")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _lds_bytes(nt):
    """k_small's LDS for nt triangles (four slots per triangle in two 16-bit
    arrays and a 32-bit one, a label byte per triangle)."""
    a16 = (8 * nt + 15) // 16 * 16
    return 4 * a16 + (nt + 15) // 16 * 16


def _corpus():
    out = [W.jittered_grid(n, seed=s) for n in (1, 2, 5, 16, 32) for s in (0, 1)]
    out += [W.jittered_grid(n, seed=40 + n, warp=True) for n in (24, 45)]
    out += [W.jittered_grid(12, seed=7, jitter=0.0)]
    out += [W.random_delaunay(n, 60 + n) for n in (4, 10, 300, 2000)]
    out += [W.scrambled(W.random_delaunay(1500, 71), 3), W.scrambled(_tall_strip(1024), 2),
            W.flat_strip(600), W.scrambled(W.flat_strip(2000), 4)]
    # either side of the workgroup's item counts (1, 2 and 4 triangles per thread)
    out += [W.flat_strip(512), W.flat_strip(513), W.flat_strip(1025)]
    for n in (12, 64):
        xy, tri = _wheel(n)
        out.append(W.Mesh(xy, tri, f"wheel{n}"))
    for name in ("p1_two_triangles_square.txt", "p3_fan_degree8.txt", "p_tie_break.txt"):
        fx = pc.load_fixture(name)
        out.append(W.Mesh(np.asarray(fx["xy"], np.int32).reshape(-1, 2), np.asarray(fx["tri"], np.int32).reshape(-1, 3),
                          name))
    xy, tri, _ = pc.grid_with_hole(40, 17, 12)
    out.append(W.Mesh(xy, tri, "hole40"))
    # loops of 62, 63, 127 and 1,001 half-edges (a loop byte holds up to 62)
    xy, tri, _, _ = pc.rising_strips([(30, True), (31, False), (63, False), (500, False)])
    out.append(W.Mesh(xy, tri, "rising_strips"))
    return out


CORPUS = _corpus()


@pytest.fixture(scope="module")
def ctxs():
    small, chain = gp.Context(0), gp.Context(0)
    chain.set_launch("small=0")
    yield small, chain
    small.close()
    chain.close()


def _run(ctx, m, flags=0):
    h = ctx.build_halfedges(m.xy, m.tri, flags)
    org, twin, nflip = h.copy()
    r = ctx.mesh(h)
    g = r.copy()
    r.free()
    h.free()
    g.update(org=org, twin=twin, nflipped=nflip)
    return g


@pytest.mark.parametrize("mesh", CORPUS, ids=[m.name for m in CORPUS])
def test_small_equals_oracle_and_chain(ctxs, mesh):
    assert mesh.nt <= 4096
    small, chain = ctxs
    say(f"[gpu] small {mesh.name}: nt={mesh.nt}")
    o = oracle.polylla(mesh.xy, mesh.tri)
    g = _run(small, mesh)
    assert_parity(g, o, mesh.name)
    c = _run(chain, mesh)
    for k in KEYS:
        assert np.array_equal(g[k], c[k]), (mesh.name, k)
    for k in ("npoly", "nloop_he", "ntips", "nmiddle", "nties"):
        assert g["info"][k] == c["info"][k], (mesh.name, k)


def test_which_form_runs():
    """Per-kernel counts of a profiling context: a mesh within the limit is
    one k_small launch; a larger one, or small=0, runs the chain."""
    with gp.Context(0, profile=True) as c:
        def launches(m):
            h = c.build_halfedges(m.xy, m.tri)
            c.kernel_reset()
            c.mesh(h).free()
            c.sync()
            h.free()
            return {k: v[1] for k, v in c.kernel_ms().items() if v[1]}
        say("[gpu] small: which form runs")
        assert launches(W.plain_small()) == {"k_small": 1}
        big = W.jittered_grid(64, seed=3)   # 8192 triangles
        got = launches(big)
        assert "k_small" not in got and got["k_label"] == 1 and got["k_relink"] == 1
        c.set_launch("small=0")
        got = launches(W.plain_small())
        assert "k_small" not in got and got["k_label"] == 1


def test_size_limit():
    """The largest meshes the form takes: 4096 triangles where the device's
    LDS per workgroup holds them, else the largest that fits 64 KiB; one
    triangle more runs the chain.  Both equal the oracle."""
    import torch
    lds = getattr(torch.cuda.get_device_properties(0), "shared_memory_per_block", 65536)
    with gp.Context(0, profile=True) as c:
        for m in (W.flat_strip(2048), W.jittered_grid(45, seed=9)):   # 4095 and 4050 triangles
            say(f"[gpu] small limit {m.name}: nt={m.nt}")
            h = c.build_halfedges(m.xy, m.tri)
            c.kernel_reset()
            r = c.mesh(h)
            g = r.copy()
            r.free()
            h.free()
            ran = {k for k, v in c.kernel_ms().items() if v[1]}
            o = oracle.polylla(m.xy, m.tri)
            for k in KEYS:
                assert np.array_equal(g[k], getattr(o, k)), (m.name, k)
            if _lds_bytes(m.nt) + 1024 <= lds:   # (the kernel's own LDS is under 1 KiB)
                assert ran == {"k_small"}, ran
        m = W.flat_strip(2049)   # 4097 triangles
        h = c.build_halfedges(m.xy, m.tri)
        c.kernel_reset()
        r = c.mesh(h)
        g = r.copy()
        r.free()
        h.free()
        assert "k_small" not in {k for k, v in c.kernel_ms().items() if v[1]}
        o = oracle.polylla(m.xy, m.tri)
        for k in KEYS:
            assert np.array_equal(g[k], getattr(o, k)), (m.name, k)


def test_small_batch_and_graph(ctxs):
    """A batch of small meshes of mixed sizes (one workgroup each, one
    launch) equals each mesh's oracle; replays of its captured graph, with
    eager work and syncs between them, equal the eager batch."""
    small, _ = ctxs
    ms = [W.jittered_grid(int(n), seed=200 + i) for i, n in enumerate([1, 3, 8, 20, 31, 45, 2, 16] * 4)]
    ms += [W.random_delaunay(1200, 300 + i) for i in range(4)]
    say(f"[gpu] small batch of {len(ms)}")
    hs = [small.build_halfedges(m.xy, m.tri) for m in ms]
    eager = []
    for r in small.mesh_batch(hs):
        eager.append(r.copy())
        r.free()
    for m, g in zip(ms, eager):
        o = oracle.polylla(m.xy, m.tri)
        for k in KEYS:
            assert np.array_equal(g[k], getattr(o, k)), (m.name, k)
    for rep in range(3):
        rs = small.mesh_batch(hs, gp.GP_GRAPH)
        for i, rr in enumerate(rs):
            got = rr.copy()
            for k in KEYS:
                assert np.array_equal(got[k], eager[i][k]), (rep, i, k)
            rr.free()
        e = small.mesh(hs[3])
        e.free()
        small.sync()
    for h in hs:
        h.free()


@pytest.mark.parametrize("mesh", [W.jittered_grid(30, seed=11, warp=True), W.scrambled(W.random_delaunay(1800, 12), 5)],
                         ids=["grid30w", "scrambled_delaunay1800"])
def test_small_compact(ctxs, mesh):
    """Compact meshes (16-bit corner and twin offsets, escapes for the rest)
    through the one-workgroup form."""
    small, _ = ctxs
    say(f"[gpu] small compact {mesh.name}")
    g = _run(small, mesh, gp.GP_COMPACT)
    assert_parity(g, oracle.polylla(mesh.xy, mesh.tri), mesh.name)
