"""Pins of the CPU oracle against what the paper and plain mathematics fix.

Hand-derived fixtures (tests/golden/*.txt, each with its derivation and the
passage it follows), closed forms on grids, brute-force Lepp regions, a
dict-based twin match, geometric middle edges, and structural invariants.
"""
import numpy as np
import pytest

import oracle
from paper_2403_14723_amd import workloads as W
from tests import polycheck as pc

FIXTURES = ["p1_two_triangles_square.txt", "p2_one_triangle.txt", "p3_fan_degree8.txt",
            "p4_fan_degree7.txt", "p_tie_break.txt"]


def polygons_as_triangle_sets(res):
    nt = len(res.org) // 3
    onloop = res.next >= 0
    comp = pc.tri_components(nt, res.twin, onloop)
    groups = {}
    for t in range(nt):
        groups.setdefault(int(comp[t]), []).append(t)
    return sorted(sorted(g) for g in groups.values())


@pytest.mark.parametrize("name", FIXTURES)
def test_fixture(name):
    fx = pc.load_fixture(name)
    res = oracle.polylla(fx["xy"], fx["tri"])
    exp = fx["expect"]
    for key in ("npoly", "ntips", "nterminal", "nmiddle", "nflipped", "nties"):
        if key in exp:
            assert res.stats[key] == exp[key], key
    for key, arr in (("next", res.next), ("prev", res.prev), ("seeds", res.seeds),
                     ("loop_off", res.loop_off), ("loop_he", res.loop_he)):
        if key in exp:
            assert list(arr) == exp[key], key
    if fx["polygons"]:
        assert polygons_as_triangle_sets(res) == fx["polygons"]
    pc.check_output(fx["xy"], res.org, res.twin, res.next, res.prev, res.seeds,
                    res.loop_off, res.loop_he)


def test_middle_edge_direction_fixture_is_geometric():
    """P4: the middle edge found by the oracle is the floor(d/2)-th neighbour
    clockwise by angle from the tip's frontier neighbour."""
    fx = pc.load_fixture("p4_fan_degree7.txt")
    res = oracle.polylla(fx["xy"], fx["tri"])
    tm = pc.tips_and_middles_geometric(fx["xy"].astype(np.int64), res.org, res.twin,
                                       res.frontier.astype(bool))
    assert tm == [(0, 5)]  # tip v=0, middle edge to s4 = vertex 5


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8, 13])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_unjittered_grid_closed_form(m, seed):
    """P5: on an unjittered grid the diagonal is the strict longest edge of
    both triangles of its cell, so every cell is one quadrilateral, whatever
    the diagonals: P = m^2, 4m^2 loop half-edges, no tips, 2m(m+1) frontier
    edges.  This matches the zero repair time on every grid row of Table 1
    and the appendix grid table."""
    mesh = W.jittered_grid(m, seed=seed, jitter=0.0)
    res = oracle.polylla(mesh.xy, mesh.tri)
    assert res.stats["npoly"] == m * m
    assert res.stats["nloop_he"] == 4 * m * m
    assert res.stats["ntips"] == 0
    info = pc.check_output(mesh.xy, res.org, res.twin, res.next, res.prev, res.seeds,
                           res.loop_off, res.loop_he)
    assert info["E"] == 2 * m * (m + 1)
    assert info["total_area2"] == 2 * (m * (W.DOMAIN // m)) ** 2


@pytest.mark.parametrize("n", [4, 9, 30, 100, 1000])
def test_paper_grid_generator(n):
    """P5 on the paper's own grid generator (Algorithm 15), whose triangles
    are clockwise and must be re-oriented: (s-1)^2 quadrilaterals."""
    xy, tri = pc.paper_grid(n)
    s = int(np.sqrt(n))
    res = oracle.polylla(xy, tri)
    assert res.stats["nflipped"] == len(tri)
    assert res.stats["npoly"] == (s - 1) ** 2
    assert res.stats["ntips"] == 0
    pc.check_output(xy, res.org, res.twin, res.next, res.prev, res.seeds, res.loop_off,
                    res.loop_he)


def _meshes_small():
    out = []
    for n in (2, 3, 5, 8, 16, 33):
        for seed in range(4):
            out.append(W.jittered_grid(n, seed=seed))
    for seed in range(3):
        out.append(W.jittered_grid(24, seed=100 + seed, warp=True))
    for npts, seed in ((30, 1), (200, 2), (1500, 3), (4000, 4)):
        out.append(W.random_delaunay(npts, seed))
    return out


SMALL = _meshes_small()


@pytest.mark.parametrize("mesh", SMALL, ids=[m.name for m in SMALL])
def test_twins_match_dict(mesh):
    """P8: twins from the sorted-key build equal a dict lookup of the
    reversed directed edge, and twin is an involution."""
    org, twin, _ = oracle.build(mesh.xy, mesh.tri)
    assert np.array_equal(twin, pc.twins_by_dict(org))
    inter = twin >= 0
    assert np.array_equal(twin[twin[inter]], np.nonzero(inter)[0])


@pytest.mark.parametrize("mesh", SMALL, ids=[m.name for m in SMALL])
def test_lepp_regions_bruteforce(mesh):
    """P6: regions from Lepp walks (Definitions 1-2) equal the components of
    triangles joined across non-frontier edges, with one terminal edge each;
    after the repair, components across non-frontier edges correspond one to
    one with the output loops."""
    res = oracle.polylla(mesh.xy, mesh.tri)
    nt = mesh.nt
    term = pc.lepp_terminal(mesh.xy, res.org, res.twin)
    comp = pc.tri_components(nt, res.twin, res.frontier.astype(bool))
    assert pc.same_partition(term, comp)
    assert len(np.unique(term)) == res.stats["nterminal"]
    # the label-phase frontier is "longest edge of neither side, or boundary"
    L = pc.longest_local(mesh.xy, res.org, res.twin)
    is_long = np.zeros(3 * nt, bool)
    is_long[3 * np.arange(nt) + L] = True
    tw = res.twin
    expect_f = (tw < 0) | (~is_long & ~is_long[np.where(tw >= 0, tw, 0)])
    assert np.array_equal(res.frontier.astype(bool), expect_f)
    assert np.array_equal(res.longest.astype(bool), is_long)
    info = pc.check_output(mesh.xy, res.org, res.twin, res.next, res.prev, res.seeds,
                           res.loop_off, res.loop_he)
    assert info["P"] == res.stats["nterminal"] + res.stats["nmiddle"]


@pytest.mark.parametrize("mesh", SMALL, ids=[m.name for m in SMALL])
def test_middle_edges_geometric(mesh):
    """The edges added by the repair are exactly the middle edges of the
    barrier tips, found by angular order around each tip."""
    res = oracle.polylla(mesh.xy, mesh.tri)
    tm = pc.tips_and_middles_geometric(mesh.xy.astype(np.int64), res.org, res.twin,
                                       res.frontier.astype(bool))
    assert len(tm) == res.stats["ntips"]
    added = (res.frontier_rep.astype(bool)) & ~(res.frontier.astype(bool))
    tgt = res.org[pc.nxt(np.arange(len(res.org)))]
    got = {tuple(sorted((int(res.org[h]), int(tgt[h])))) for h in np.nonzero(added)[0]}
    want = {tuple(sorted(p)) for p in tm}
    assert got == want
    assert len(want) == res.stats["nmiddle"]


def test_delaunay_has_tips():
    """The general-position input really exercises the repair."""
    res = oracle.polylla(*(lambda m: (m.xy, m.tri))(W.random_delaunay(4000, 4)))
    assert res.stats["ntips"] > 20


@pytest.mark.parametrize("seed", range(6))
def test_permutation_metamorphic(seed):
    """P10: on a tie-free input, renumbering triangles and rotating their
    corners gives the same polygons as sets of triangles."""
    mesh = W.random_delaunay(800, 50 + seed) if seed % 2 else W.jittered_grid(12, seed=seed)
    base = oracle.polylla(mesh.xy, mesh.tri)
    assert base.stats["nties"] == 0
    rng = np.random.default_rng(seed)
    perm = rng.permutation(mesh.nt)
    rot = rng.integers(0, 3, mesh.nt)
    tri2 = np.stack([np.roll(mesh.tri[p], -r) for p, r in zip(perm, rot)])
    res2 = oracle.polylla(mesh.xy, tri2)
    assert res2.stats["npoly"] == base.stats["npoly"]
    a = polygons_as_triangle_sets(base)
    b = sorted(sorted(int(perm[t]) for t in g) for g in polygons_as_triangle_sets(res2))
    assert a == b


def test_domain_area_full_square():
    """Loop areas add up to the exact domain area, 2 * (2^20)^2 doubled."""
    mesh = W.jittered_grid(64, seed=9, warp=True)
    res = oracle.polylla(mesh.xy, mesh.tri)
    info = pc.check_output(mesh.xy, res.org, res.twin, res.next, res.prev, res.seeds,
                           res.loop_off, res.loop_he)
    assert info["total_area2"] == 2 * (1 << 40)


# ---------------------------------------------------------------------------
# error paths
# ---------------------------------------------------------------------------

def _expect_err(xy, tri, code):
    with pytest.raises(oracle.OracleError) as e:
        oracle.polylla(np.array(xy), np.array(tri))
    assert e.value.code == code


def test_err_nonmanifold_edge():
    xy = [[0, 10], [10, 10], [5, 15], [5, 5], [5, 19]]
    _expect_err(xy, [[0, 1, 2], [1, 0, 3], [0, 1, 4]], oracle.ORC_ENONMANIFOLD)


def test_err_duplicate_triangle():
    xy = [[0, 0], [10, 0], [5, 5]]
    _expect_err(xy, [[0, 1, 2], [0, 1, 2]], oracle.ORC_ENONMANIFOLD)


def test_err_zero_area():
    _expect_err([[0, 0], [1, 1], [2, 2]], [[0, 1, 2]], oracle.ORC_EDEGEN)


def test_err_index_out_of_range():
    _expect_err([[0, 0], [1, 0], [0, 1]], [[0, 1, 3]], oracle.ORC_EINVAL)
    _expect_err([[0, 0], [1, 0], [0, 1]], [[0, -1, 2]], oracle.ORC_EINVAL)


def test_err_coordinate_range():
    oracle.polylla(np.array([[0, 0], [1 << 30, 0], [0, 1]]), np.array([[0, 1, 2]]))  # at the limit: fine
    _expect_err([[0, 0], [(1 << 30) + 1, 0], [0, 1]], [[0, 1, 2]], oracle.ORC_ERANGE)
    _expect_err([[-1, 0], [1, 0], [0, 1]], [[0, 1, 2]], oracle.ORC_ERANGE)


def test_err_too_many_triangles():
    import ctypes
    lib = oracle._load()
    buf = (ctypes.c_int32 * 6)()
    nt = (1 << 31) // 3 + 1
    rc = lib.orc_build(buf, 1, buf, nt, buf, buf, None)
    assert rc == oracle.ORC_ERANGE


def test_empty_and_unused_vertices():
    res = oracle.polylla(np.zeros((0, 2), np.int32), np.zeros((0, 3), np.int32))
    assert res.stats["npoly"] == 0 and len(res.loop_off) == 1
    # a vertex that no triangle uses is allowed
    xy = np.array([[0, 0], [10, 0], [0, 10], [77, 77]], np.int32)
    res = oracle.polylla(xy, np.array([[0, 1, 2]], np.int32))
    assert res.stats["npoly"] == 1


@pytest.mark.parametrize("n", [1, 2, 7, 500])
def test_flat_strip_closed_form(n):
    """Flat triangles whose longest edges all lie on the boundary, where a
    Lepp ends at once (Section 3.1, Definitions 1-2; terminal edges may be
    border edges), and whose shared sides are the longest edge of neither
    neighbour, so frontier (Definition 3): each triangle is a terminal-edge
    region and a polygon of its own, and its loop is its three half-edges in
    order."""
    m = W.flat_strip(n)
    o = oracle.polylla(m.xy, m.tri)
    T = m.nt
    h = np.arange(3 * T)
    assert T == 2 * n - 1
    assert o.stats["npoly"] == T and o.stats["nloop_he"] == 3 * T and o.stats["ntips"] == 0
    np.testing.assert_array_equal(o.seeds, 3 * np.arange(T))
    np.testing.assert_array_equal(o.loop_off, 3 * np.arange(T + 1))
    np.testing.assert_array_equal(o.loop_he, h)
    np.testing.assert_array_equal(o.next, 3 * (h // 3) + (h % 3 + 1) % 3)
    np.testing.assert_array_equal(o.prev, 3 * (h // 3) + (h % 3 + 2) % 3)


@pytest.mark.parametrize("case", ["hole", "two"])
def test_hole_and_two_components(case):
    """Domains that are not disks: a grid with a hole (an inner boundary
    loop) and two disjoint grids.  Every structural invariant holds, with
    V - E + P equal to the domain's Euler characteristic (0 and 2)."""
    xy, tri, chi = pc.grid_with_hole(24, 7, 6) if case == "hole" else pc.two_grids(12, 17, 8)
    o = oracle.polylla(xy, tri)
    pc.check_output(xy, o.org, o.twin, o.next, o.prev, o.seeds, o.loop_off, o.loop_he, chi=chi)


@pytest.mark.parametrize("seed", range(3))
def test_scrambled_is_the_same_triangulation(seed):
    """The scrambling input generator keeps the triangulation: the same
    triangles as sets of points, and on a tie-free mesh the oracle finds as
    many polygons, with every structural invariant intact."""
    m = W.random_delaunay(1500, 60 + seed)
    s = W.scrambled(m, seed)
    assert s.nv == m.nv and s.nt == m.nt
    key = lambda xy, tri: sorted(tuple(sorted(map(tuple, xy[t].tolist()))) for t in tri)
    assert key(m.xy, m.tri) == key(s.xy, s.tri)
    a, b = oracle.polylla(m.xy, m.tri), oracle.polylla(s.xy, s.tri)
    assert a.stats["nties"] == 0 and 0 < b.stats["nflipped"] < s.nt
    assert b.stats["npoly"] == a.stats["npoly"] and b.stats["nloop_he"] == a.stats["nloop_he"]
    pc.check_output(s.xy, b.org, b.twin, b.next, b.prev, b.seeds, b.loop_off, b.loop_he)


def test_rising_strips_one_polygon_each():
    """Closed form: a strip whose rungs grow strictly along it is one polygon
    (each inner rung is the longest edge of exactly one side, the last rung
    terminal), with its whole boundary as the loop: 2n + 1 half-edges, or
    2n + 2 when a top triangle closes it.  Loops of 62 to 66 half-edges sit
    either side of the longest length a loop byte holds (62)."""
    cases = [(30, True), (31, False), (31, True), (32, False), (32, True), (63, False), (500, False)]
    xy, tri, chi, lens = pc.rising_strips(cases)
    o = oracle.polylla(xy, tri)
    assert o.stats["npoly"] == len(cases) and o.stats["ntips"] == 0
    np.testing.assert_array_equal(np.diff(o.loop_off), lens)
    assert o.stats["nloop_he"] == sum(lens)
    pc.check_output(xy, o.org, o.twin, o.next, o.prev, o.seeds, o.loop_off, o.loop_he, chi=chi)
