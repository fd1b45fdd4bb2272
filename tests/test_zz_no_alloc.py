"""gpolylla_mesh_noalloc: the meshing run into caller-allocated device
buffers with the library's static scratch, checked element by element against
gpolylla_mesh (whose results the parity tests check against the oracle) on two
calls in a row, the second on a smaller mesh."""
import numpy as np
import pytest

import paper_2403_14723_amd as gp
from paper_2403_14723_amd import workloads as W

pytestmark = pytest.mark.gpu


def _noalloc(ctx, h, nt):
    import torch
    dev = torch.device("cuda", 0)
    nh = 3 * nt
    # filled with a sentinel so that untouched entries would show
    bufs = {k: torch.full((n,), -7, dtype=torch.int32, device=dev)
            for k, n in (("next", nh + 1), ("prev", nh + 1), ("seeds", nt + 1), ("loop_off", nt + 2),
                         ("loop_he", nh + 1))}
    counts = torch.full((8,), 99, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    out = gp.gp_result_dev(*[bufs[k].data_ptr() for k in ("next", "prev", "seeds", "loop_off", "loop_he")])
    rc = gp.gpolylla_mesh_noalloc(ctx.handle, h.handle, out, counts.data_ptr())
    assert rc == gp.GP_OK, gp.gpolylla_strerror(rc)
    ctx.sync()
    c = counts.cpu().numpy()
    return {k: v.cpu().numpy() for k, v in bufs.items()}, c


def test_noalloc_matches_mesh_on_two_calls():
    meshes = [W.plain_scale(), W.jittered_grid(96, seed=7, warp=True, name="g96w")]
    assert meshes[1].nt < meshes[0].nt
    with gp.Context(0) as ctx:
        for m in meshes:
            print(f"[noalloc] {m.name} nt={m.nt}", flush=True)
            h = ctx.build_halfedges(m.xy, m.tri)
            r = ctx.mesh(h)
            ref = r.copy()
            r.free()
            got, c = _noalloc(ctx, h, m.nt)
            info = ref["info"]
            P, Fh, nh = info["npoly"], info["nloop_he"], info["nh"]
            assert c[0] == gp.GP_OK
            assert (c[1], c[2], c[3], c[4], c[5]) == (P, Fh, info["ntips"], info["nmiddle"], info["nties"])
            assert c[6] == 0 and c[7] == 0
            np.testing.assert_array_equal(got["next"][:nh], ref["next"])
            np.testing.assert_array_equal(got["prev"][:nh], ref["prev"])
            np.testing.assert_array_equal(got["seeds"][:P], ref["seeds"])
            np.testing.assert_array_equal(got["loop_off"][:P + 1], ref["loop_off"])
            np.testing.assert_array_equal(got["loop_he"][:Fh], ref["loop_he"])
            h.free()


def test_noalloc_refuses_a_mesh_beyond_the_scratch():
    """A mesh whose scratch needs far more than the static array (8.4M
    triangles, about 450 MB of scratch against 256 MiB) is refused before any
    work is queued.  The output buffers are real and large enough anyway, so
    a refusal that did not happen would fail this test, not the device."""
    import torch
    m = W.jittered_grid(2048, seed=8, name="g2048")
    nt, nh = m.nt, 3 * m.nt
    dev = torch.device("cuda", 0)
    with gp.Context(0) as ctx:
        h = ctx.build_halfedges(m.xy, m.tri)
        bufs = [torch.empty(n, dtype=torch.int32, device=dev) for n in (nh + 1, nh + 1, nt + 1, nt + 2, nh + 1)]
        counts = torch.zeros(8, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        out = gp.gp_result_dev(*[b.data_ptr() for b in bufs])
        rc = gp.gpolylla_mesh_noalloc(ctx.handle, h.handle, out, counts.data_ptr())
        ctx.sync()
        assert rc == gp.GP_ETOOBIG
        # and the context still meshes normally afterwards
        r = ctx.mesh(h)
        assert r.info()["npoly"] > 0
        r.free()
        h.free()


def test_noalloc_argument_errors():
    with gp.Context(0) as ctx:
        m = W.plain_small()
        h = ctx.build_halfedges(m.xy, m.tri)
        out = gp.gp_result_dev(0, 0, 0, 0, 0)
        assert gp.gpolylla_mesh_noalloc(ctx.handle, h.handle, out, 0) == gp.GP_EINVAL
        h.free()
