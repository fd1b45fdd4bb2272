"""Intermediate stages of a debug run, each against what the oracle's labels
fix: the label bytes after the relink (longest edge, label-phase frontier,
seeds), next'/prev' before the repair (the turns of Section 6.5 over the
label-phase frontier, done here by brute force), the barrier tips (next'(h)
== twin(h), Section 5.2), and the label bytes after the repair (the repaired
frontier).  The final outputs still equal the oracle's."""
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
def dctx():
    c = gp.Context(0)
    c.set_debug(True)
    yield c
    c.close()


def _nxt(h):
    return h - 2 if h % 3 == 2 else h + 1


def _prv(h):
    return h + 2 if h % 3 == 0 else h - 1


def expected_stages(o):
    """Label bytes and next'/prev' before the repair, from the oracle's
    longest-edge and label-phase frontier arrays (brute-force turns)."""
    nh = len(o.twin)
    nt = nh // 3
    longest = o.longest.astype(bool)
    fr = o.frontier.astype(bool)
    L = longest.reshape(nt, 3).argmax(axis=1)
    assert (longest.reshape(nt, 3).sum(axis=1) == 1).all()
    h_l = 3 * np.arange(nt) + L
    g = o.twin[h_l]
    seed = (g < 0) | ((g >= 0) & longest[np.maximum(g, 0)] & (h_l < g))
    tflag = (L | (fr.reshape(nt, 3) * np.array([4, 8, 16])).sum(axis=1) | np.where(seed, 32, 0)).astype(np.uint8)
    nx = np.full(nh, -1, np.int64)
    pv = np.full(nh, -1, np.int64)
    for h in np.nonzero(fr)[0]:
        c = _nxt(h)
        while not fr[c]:
            c = _nxt(o.twin[c])
        nx[h] = c
        c = _prv(h)
        while not fr[c]:
            c = _prv(o.twin[c])
        pv[h] = c
    tips = np.nonzero(fr & (nx == o.twin))[0]
    return tflag, nx, pv, tips


CASES = [W.jittered_grid(30, seed=1101), W.random_delaunay(4000, 1102), W.random_delaunay(15000, 1103),
         W.scrambled(W.random_delaunay(3000, 1104), 9), W.flat_strip(300)]


@pytest.mark.parametrize("mesh", CASES, ids=[m.name for m in CASES])
def test_intermediate_stages(dctx, mesh):
    say(f"[gpu] debug stages {mesh.name}")
    o = oracle.polylla(mesh.xy, mesh.tri)
    h = dctx.build_halfedges(mesh.xy, mesh.tri)
    r = dctx.mesh(h)
    d = r.debug()
    g = r.copy()
    org, twin, nflip = h.copy()
    g.update(org=org, twin=twin, nflipped=nflip)
    r.free()
    h.free()
    assert_parity(g, o, "debug:" + mesh.name)
    tflag, nx, pv, tips = expected_stages(o)
    assert np.array_equal(d["tflag_relink"], tflag)
    assert np.array_equal(d["next_relink"], nx)
    assert np.array_equal(d["prev_relink"], pv)
    assert np.array_equal(d["tips"], tips) and d["ntips"] == len(tips) == g["info"]["ntips"]
    nt = mesh.nt
    rep = (o.frontier_rep.astype(np.uint8).reshape(nt, 3) * np.array([4, 8, 16], np.uint8)).sum(axis=1)
    assert np.array_equal(d["tflag_final"] & 0x1c, rep.astype(np.uint8))
    assert np.array_equal(d["tflag_final"] & 3, tflag & 3)


def test_debug_in_a_batch_and_off(dctx):
    """Each result of a batched debug run gets its own mesh's stages and tips;
    a run without debug has none to give."""
    ms = [W.random_delaunay(2000, 1110), W.jittered_grid(12, seed=1111), W.random_delaunay(5000, 1112)]
    hs = [dctx.build_halfedges(m.xy, m.tri) for m in ms]
    rs = dctx.mesh_batch(hs)
    for m, r in zip(ms, rs):
        o = oracle.polylla(m.xy, m.tri)
        tflag, nx, pv, tips = expected_stages(o)
        d = r.debug()
        assert np.array_equal(d["tflag_relink"], tflag) and np.array_equal(d["next_relink"], nx)
        assert np.array_equal(d["tips"], tips)
        r.free()
    for h in hs:
        h.free()
    with gp.Context(0) as c:
        m = ms[1]
        h = c.build_halfedges(m.xy, m.tri)
        r = c.mesh(h)
        with pytest.raises(gp.GPolyllaError) as e:
            r.debug()
        assert e.value.code == gp.GP_EINVAL
        r.free()
        h.free()
