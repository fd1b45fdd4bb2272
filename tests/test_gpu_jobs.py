"""Host-to-host jobs with overlapped copies (gpolylla_mesh_jobs): every job's
outputs equal the oracle's element by element (integer outputs: tolerance
zero), with full outputs and loops only, across group boundaries, with a
failing job among good ones and an empty one."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import paper_2403_14723_amd as gp
from paper_2403_14723_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gp.Context(0)
    yield c
    c.close()


def _job(m, loops_only=False):
    nt = m.nt
    bufs = {"xy": np.ascontiguousarray(m.xy, dtype=np.int32), "tri": np.ascontiguousarray(m.tri, dtype=np.int32),
            "seeds": np.full(max(nt, 1), -7, np.int32), "loop_off": np.full(nt + 1, -7, np.int32),
            "loop_he": np.full(max(3 * nt, 1), -7, np.int32)}
    if not loops_only:
        bufs["next"] = np.full(max(3 * nt, 1), -7, np.int32)
        bufs["prev"] = np.full(max(3 * nt, 1), -7, np.int32)
    j = gp.gp_job()
    j.xy, j.nv = bufs["xy"].ctypes.data, m.nv
    j.tri, j.nt = bufs["tri"].ctypes.data, nt
    for k in ("next", "prev", "seeds", "loop_off", "loop_he"):
        setattr(j, k, bufs[k].ctypes.data if k in bufs else None)
    return j, bufs


def _check(j, bufs, m, name):
    assert j.status == gp.GP_OK, (name, j.status)
    o = oracle.polylla(m.xy, m.tri)
    P, F = j.npoly, j.nloop_he
    assert P == len(o.seeds) and F == len(o.loop_he), name
    assert np.array_equal(bufs["seeds"][:P], o.seeds), name
    assert np.array_equal(bufs["loop_off"][:P + 1], o.loop_off), name
    assert np.array_equal(bufs["loop_he"][:F], o.loop_he), name
    if "next" in bufs:
        assert np.array_equal(bufs["next"][:3 * m.nt], o.next), name
        assert np.array_equal(bufs["prev"][:3 * m.nt], o.prev), name


def _meshes():
    return [W.jittered_grid(40, seed=801), W.jittered_grid(7, seed=802, warp=True),
            W.random_delaunay(3000, 803), W.jittered_grid(150, seed=804, warp=True),
            W.jittered_grid(1, seed=805), W.random_delaunay(20000, 806), W.jittered_grid(99, seed=807)]


@pytest.mark.parametrize("loops_only", [False, True])
@pytest.mark.parametrize("group", [0, 5000, 60000])
def test_jobs_match_oracle(ctx, loops_only, group):
    ms = _meshes()
    say(f"[gpu] jobs: {len(ms)} meshes, group {group}, loops only {loops_only}")
    built = [_job(m, loops_only) for m in ms]
    arr = (gp.gp_job * len(ms))(*[b[0] for b in built])
    rc = gp.gpolylla_mesh_jobs(ctx.handle, arr, group)
    assert rc == gp.GP_OK, rc
    for k, m in enumerate(ms):
        _check(arr[k], built[k][1], m, f"{m.name} group={group}")


def test_jobs_with_a_failing_and_an_empty_job(ctx):
    """A job whose input the build rejects gets that error as its status; the
    jobs around it (same group and next group) still come back whole; an
    empty triangulation gives no polygons."""
    good = [W.jittered_grid(30, seed=811), W.jittered_grid(12, seed=812, warp=True)]
    bad = W.jittered_grid(5, seed=813)
    tri = bad.tri.copy()
    tri[3] = tri[2]   # a repeated triangle: the same directed edges twice
    bad = W.Mesh(bad.xy, tri, bad.name + "_dup")
    want_bad = None
    try:
        oracle.polylla(bad.xy, bad.tri)
    except oracle.OracleError as e:
        want_bad = e.code
    assert want_bad is not None
    empty = W.Mesh(np.zeros((3, 2), np.int32), np.zeros((0, 3), np.int32), "empty")
    ms = [good[0], bad, empty, good[1]]
    say("[gpu] jobs: a failing and an empty job")
    built = [_job(m) for m in ms]
    arr = (gp.gp_job * len(ms))(*[b[0] for b in built])
    rc = gp.gpolylla_mesh_jobs(ctx.handle, arr, 2000)
    assert rc == want_bad
    assert arr[1].status == want_bad
    assert arr[2].status == gp.GP_OK and arr[2].npoly == 0 and arr[2].nloop_he == 0
    assert built[2][1]["loop_off"][0] == 0
    for k in (0, 3):
        _check(arr[k], built[k][1], ms[k], ms[k].name)


def test_jobs_argument_errors(ctx):
    m = W.jittered_grid(4, seed=821)
    j, bufs = _job(m)
    j.prev = None   # next without prev
    arr = (gp.gp_job * 1)(j)
    assert gp.gpolylla_mesh_jobs(ctx.handle, arr, 0) == gp.GP_EINVAL
    j2, bufs2 = _job(m)
    arr2 = (gp.gp_job * 1)(j2)
    assert gp.gpolylla_mesh_jobs(ctx.handle, arr2, 0, flags=0x100) == gp.GP_EINVAL
    assert gp.gpolylla_mesh_jobs(ctx.handle, (gp.gp_job * 0)(), 0) == gp.GP_OK


def _small_jobs_list():
    """Jobs that all fit one workgroup (at most 4,096 triangles and 4,096
    vertices): the list goes through the packed path, one build-and-mesh
    launch per group."""
    from tests.test_gpu_parity import _tall_strip, _wheel
    ms = [W.jittered_grid(n, seed=830 + n, warp=(n % 2 == 0)) for n in (1, 2, 5, 16, 32, 45)]
    ms += [W.random_delaunay(n, 840 + n) for n in (4, 50, 1000, 2000)]
    ms += [W.scrambled(W.random_delaunay(1500, 851), 3), W.scrambled(_tall_strip(1024), 2), W.flat_strip(700)]
    xy, tri = _wheel(40)
    ms.append(W.Mesh(xy, tri, "wheel40"))
    return ms


@pytest.mark.parametrize("loops_only", [False, True])
@pytest.mark.parametrize("group", [0, 3000])
def test_small_jobs_packed_match_oracle(ctx, loops_only, group):
    ms = _small_jobs_list()
    assert all(m.nt <= 4096 and m.nv <= 4096 for m in ms)
    say(f"[gpu] small jobs: {len(ms)} meshes, group {group}, loops only {loops_only}")
    built = [_job(m, loops_only) for m in ms]
    arr = (gp.gp_job * len(ms))(*[b[0] for b in built])
    rc = gp.gpolylla_mesh_jobs(ctx.handle, arr, group)
    assert rc == gp.GP_OK, rc
    for k, m in enumerate(ms):
        _check(arr[k], built[k][1], m, f"{m.name} group={group}")


def test_small_jobs_packed_errors(ctx):
    """Each build error of the staged build, in a packed group beside good
    jobs: the same status as gpolylla_build_halfedges and the oracle give,
    including a job with several errors (the lowest-ranked is reported: a
    coordinate before a bad triangle, the lowest bad triangle before a later
    one) and an empty job."""
    cases = {
        "nonmanifold": ([[0, 10], [10, 10], [5, 15], [5, 5], [5, 19]], [[0, 1, 2], [1, 0, 3], [0, 1, 4]]),
        "duplicate": ([[0, 0], [10, 0], [5, 5]], [[0, 1, 2], [0, 1, 2]]),
        "zero_area": ([[0, 0], [1, 1], [2, 2]], [[0, 1, 2]]),
        "index": ([[0, 0], [1, 0], [0, 1]], [[0, 1, 3]]),
        "coord": ([[0, 0], [(1 << 30) + 1, 0], [0, 1]], [[0, 1, 2]]),
        "coord_and_index": ([[0, 0], [1, 0], [0, 1], [-5, 0]], [[0, 1, 7], [0, 1, 2]]),
        "zero_area_then_index": ([[0, 0], [1, 1], [2, 2], [0, 5]], [[0, 1, 2], [0, 1, 9]]),
        "index_then_zero_area": ([[0, 0], [1, 1], [2, 2], [0, 5]], [[0, 1, 9], [0, 1, 2]]),
    }
    bad = [W.Mesh(np.array(x, np.int32), np.array(t, np.int32), name) for name, (x, t) in cases.items()]
    good = [W.jittered_grid(9, seed=861), W.random_delaunay(300, 862)]
    empty = W.Mesh(np.zeros((3, 2), np.int32), np.zeros((0, 3), np.int32), "empty")
    ms = [good[0]] + bad + [empty, good[1]]
    want = {}
    for m in bad:
        with pytest.raises(oracle.OracleError) as eo:
            oracle.polylla(m.xy, m.tri)
        with pytest.raises(gp.GPolyllaError) as eg:
            ctx.build_halfedges(m.xy, m.tri)
        assert eg.value.code == eo.value.code, m.name
        want[m.name] = eo.value.code
    say("[gpu] small jobs: build errors in a packed group")
    built = [_job(m) for m in ms]
    arr = (gp.gp_job * len(ms))(*[b[0] for b in built])
    rc = gp.gpolylla_mesh_jobs(ctx.handle, arr, 0)
    assert rc == want[bad[0].name]
    for k, m in enumerate(ms):
        if m.name in want:
            assert arr[k].status == want[m.name], (m.name, arr[k].status)
    assert arr[len(ms) - 2].status == gp.GP_OK and arr[len(ms) - 2].npoly == 0
    assert built[len(ms) - 2][1]["loop_off"][0] == 0
    for k in (0, len(ms) - 1):
        _check(arr[k], built[k][1], ms[k], ms[k].name)
