"""The halo that splitting one mesh over several devices needs, checked on the
CPU with the oracle.

A device that owns a set P of triangles (its band) and also holds every
triangle within k vertex rings of P meshes its copy on its own.  For the
half-edges of P the labels, the repaired frontier and next'/prev' must then be
those of the whole mesh, so that only loops cut by a band boundary need a
stitching step.  The repair (Section 6.4) adds the middle edge of each barrier
tip, and next'/prev' (Section 6.5) turn around the target vertex, so an edge
incident to a band vertex can change because of a tip one ring further out:
two rings are enough and one is not.
"""
import numpy as np
import pytest

import oracle
from paper_2403_14723_amd import workloads as W


def _grow(tri, sel):
    """Triangles that share a vertex with a selected one."""
    on = np.zeros(int(tri.max()) + 1, bool)
    on[tri[sel].ravel()] = True
    return on[tri].any(1)


def _band_mismatches(m, full, proper, rings):
    """Half-edges of the proper triangles whose repaired frontier bit, next' or
    prev' differ between the whole mesh and the band with `rings` rings."""
    keep = proper.copy()
    for _ in range(rings):
        keep = _grow(m.tri, keep)
    ids = np.nonzero(keep)[0]
    sub = oracle.polylla(m.xy, m.tri[ids])   # the unused vertices stay: allowed
    to_full = (3 * ids[:, None] + np.arange(3)).ravel()
    local = np.nonzero(proper[ids])[0]
    sh = (3 * local[:, None] + np.arange(3)).ravel()
    fh = to_full[sh]
    nx = np.where(sub.next[sh] >= 0, to_full[np.maximum(sub.next[sh], 0)], -1)
    pv = np.where(sub.prev[sh] >= 0, to_full[np.maximum(sub.prev[sh], 0)], -1)
    return int((nx != full.next[fh]).sum() + (pv != full.prev[fh]).sum()
               + (sub.frontier_rep[sh] != full.frontier_rep[fh]).sum())


def _slab(m, lo, hi):
    cx = m.xy[m.tri, 0].astype(np.float64).mean(1)
    return (cx >= lo * W.DOMAIN) & (cx < hi * W.DOMAIN)


@pytest.mark.parametrize("seed", range(8))
def test_two_rings_reproduce_the_whole_mesh(seed):
    m = W.random_delaunay(3000, 300 + seed)
    full = oracle.polylla(m.xy, m.tri)
    assert full.stats["ntips"] > 50   # the repair is exercised near every cut
    for lo, hi in ((0.0, 0.3), (0.3, 0.6), (0.6, 1.01)):
        assert _band_mismatches(m, full, _slab(m, lo, hi), 2) == 0


def test_one_ring_is_not_enough():
    # Delaunay of 3000 points, seed 302: a barrier tip one ring outside the
    # slab adds a middle edge at a slab vertex, which a one-ring copy misses
    m = W.random_delaunay(3000, 302)
    full = oracle.polylla(m.xy, m.tri)
    proper = _slab(m, 0.3, 0.6)
    assert _band_mismatches(m, full, proper, 0) > 100
    assert _band_mismatches(m, full, proper, 1) > 0
    assert _band_mismatches(m, full, proper, 2) == 0


@pytest.mark.parametrize("band", range(4))
def test_grid_band_rows_match_whole_grid(band):
    # grid_band's two halo rows are two vertex rings: the band proper's
    # half-edges of the band mesh equal the whole grid's, shifted by the cut
    n, nb = 48, 4
    m = W.jittered_grid(n, seed=40 + band, warp=True)
    full = oracle.polylla(m.xy, m.tri)
    b = W.grid_band(m, n, band, nb)
    sub = oracle.polylla(b.xy, b.tri)
    rows = n // nb
    j0 = max(0, band * rows - 2)
    off = 6 * n * j0
    lo, hi = 6 * n * band * rows - off, 6 * n * (band + 1) * rows - off
    s = slice(lo, hi)
    f = slice(lo + off, hi + off)
    assert b.nt == 2 * n * (min(n, (band + 1) * rows + 2) - j0)
    np.testing.assert_array_equal(np.where(sub.next[s] >= 0, sub.next[s] + off, -1), full.next[f])
    np.testing.assert_array_equal(np.where(sub.prev[s] >= 0, sub.prev[s] + off, -1), full.prev[f])
    np.testing.assert_array_equal(sub.frontier_rep[s], full.frontier_rep[f])
