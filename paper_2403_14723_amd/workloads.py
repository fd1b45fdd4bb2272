"""Seeded synthetic triangulations: the inputs that both the HIP path and the
oracle consume.

This module holds only input recipes (coordinates and triangle index triples);
none of the meshing arithmetic lives here.  Every random draw comes from
splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) applied to a counter built from (seed, stream,
index), so an array element never depends on how many other elements were
drawn before it.

The workloads follow the shape of the paper's Grid meshes (Section 7.1,
Algorithm 15: a square grid of points, each cell split into two triangles) at
sizes comparable to its Table 1 / appendix rows.  Its Random (Delaunay) meshes
came from an external Delaunay code that is not available: jitter, random
diagonals and a smooth warp bring irregularity to the grids, and
random_delaunay (scipy's Qhull on seeded random points) stands in for the
Random meshes themselves.

Recipe (all coordinates are integers in [0, 2**20]):
  * n x n cells of side c = floor(2**20 / n); vertex (i, j) has id j*(n+1)+i and
    nominal position (i*c, j*c);
  * integer jitter uniform in [-J, J], J = floor(0.2*c); boundary vertices
    move only along the boundary and the four corners stay fixed, so the
    domain stays the exact square;
  * each cell draws one bit b (p = 1/2): b = 0 gives (v00,v10,v11),
    (v00,v11,v01); b = 1 gives (v00,v10,v01), (v10,v11,v01); cell (i, j)
    owns triangles 2*(j*n+i) and 2*(j*n+i)+1;
  * optional warp: the sum of 8 Gaussian bumps of amplitude 0.35*c, centres
    uniform in the domain, directions uniform on the circle, widths
    log-uniform in [4, 64] cells, evaluated at the nominal position, each
    component capped at 0.35*c (this only acts where bumps overlap), rounded,
    and on the boundary restricted to the tangential component.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

DOMAIN = 1 << 20

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_GOLD = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)

# stream tags: each kind of draw has its own counter space
_S_JX, _S_JY, _S_DIAG, _S_WARP, _S_MESH, _S_REQ, _S_PTS, _S_SCR = 1, 2, 3, 4, 5, 6, 7, 8


def splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser on a uint64 array (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = (x.astype(np.uint64) + _GOLD) & _M64
        z = ((z ^ (z >> np.uint64(30))) * _MIX1) & _M64
        z = ((z ^ (z >> np.uint64(27))) * _MIX2) & _M64
        return z ^ (z >> np.uint64(31))


def _counter(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    if not (0 <= seed < (1 << 20)):
        raise ValueError("seed must be in [0, 2**20)")
    base = np.uint64(((seed << 8) | stream) << 36)
    return splitmix64(base ^ idx.astype(np.uint64))


def uniform_int(seed: int, stream: int, idx: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """Integers uniform in [lo, hi] (inclusive), one per counter value."""
    span = np.uint64(hi - lo + 1)
    return (_counter(seed, stream, idx) % span).astype(np.int64) + lo


def uniform01(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Doubles uniform in [0, 1) from the top 53 bits."""
    return (_counter(seed, stream, idx) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


@dataclass(frozen=True)
class Mesh:
    """A triangulation: xy is int32 (V, 2), tri is int32 (T, 3)."""
    xy: np.ndarray
    tri: np.ndarray
    name: str = ""

    @property
    def nv(self) -> int:
        return int(self.xy.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tri.shape[0])


def grid_triangles(n: int, diag: np.ndarray) -> np.ndarray:
    """Two triangles per cell of an n x n grid, split by the per-cell bit."""
    j, i = np.meshgrid(np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int64), indexing="ij")
    v00 = j * (n + 1) + i
    v10 = v00 + 1
    v01 = v00 + (n + 1)
    v11 = v01 + 1
    b = diag.reshape(n, n).astype(bool)
    t0 = np.where(b[..., None], np.stack([v00, v10, v01], -1), np.stack([v00, v10, v11], -1))
    t1 = np.where(b[..., None], np.stack([v10, v11, v01], -1), np.stack([v00, v11, v01], -1))
    tri = np.stack([t0, t1], axis=2).reshape(-1, 3)
    return np.ascontiguousarray(tri.astype(np.int32))


def _warp_field(seed: int, px: np.ndarray, py: np.ndarray, c: float, nbumps: int = 8,
                amp: float = 0.35) -> tuple[np.ndarray, np.ndarray]:
    k = np.arange(nbumps * 8, dtype=np.uint64)
    r = uniform01(seed, _S_WARP, k).reshape(nbumps, 8)
    cx = r[:, 0] * DOMAIN
    cy = r[:, 1] * DOMAIN
    ang = r[:, 2] * (2.0 * math.pi)
    sig = np.exp(np.log(4.0) + r[:, 3] * (np.log(64.0) - np.log(4.0))) * c
    dx = np.zeros(px.shape, np.float64)
    dy = np.zeros(px.shape, np.float64)
    for b in range(nbumps):
        g = np.exp(-((px - cx[b]) ** 2 + (py - cy[b]) ** 2) / (2.0 * sig[b] ** 2))
        dx += amp * c * math.cos(ang[b]) * g
        dy += amp * c * math.sin(ang[b]) * g
    return dx, dy


def jittered_grid(n: int, seed: int, jitter: float = 0.2, warp: bool = False,
                  name: str = "") -> Mesh:
    """n x n cell grid with the recipe in the module docstring.  The cell side
    is c = floor(2**20 / n) and the domain is [0, n*c]^2 (the full [0, 2**20]^2
    when n divides 2**20)."""
    if not (1 <= n <= 1 << 15):
        raise ValueError("n must be in [1, 32768]")
    c = DOMAIN // n
    J = int(math.floor(jitter * c))
    nv = (n + 1) * (n + 1)
    idx = np.arange(nv, dtype=np.uint64)
    jj, ii = np.divmod(np.arange(nv, dtype=np.int64), n + 1)
    x = ii * c
    y = jj * c
    dx = uniform_int(seed, _S_JX, idx, -J, J) if J > 0 else np.zeros(nv, np.int64)
    dy = uniform_int(seed, _S_JY, idx, -J, J) if J > 0 else np.zeros(nv, np.int64)
    if warp:
        wx = np.empty(nv, np.float64)
        wy = np.empty(nv, np.float64)
        step = 1 << 22
        for s in range(0, nv, step):
            a, b = _warp_field(seed, x[s:s + step].astype(np.float64),
                               y[s:s + step].astype(np.float64), float(c))
            wx[s:s + step] = a
            wy[s:s + step] = b
        # where bumps overlap their sum could exceed one bump's amplitude;
        # capping each component at 0.35*c keeps every vertex more than half
        # a cell from the domain side and from the corners
        cap = 0.35 * c
        dx = dx + np.rint(np.clip(wx, -cap, cap)).astype(np.int64)
        dy = dy + np.rint(np.clip(wy, -cap, cap)).astype(np.int64)
    dx = np.where((ii == 0) | (ii == n), 0, dx)   # left/right boundary: x pinned
    dy = np.where((jj == 0) | (jj == n), 0, dy)   # bottom/top boundary: y pinned
    hi = n * c
    x = np.clip(x + dx, 0, hi)
    y = np.clip(y + dy, 0, hi)
    xy = np.ascontiguousarray(np.stack([x, y], -1).astype(np.int32))
    diag = uniform_int(seed, _S_DIAG, np.arange(n * n, dtype=np.uint64), 0, 1)
    return Mesh(xy, grid_triangles(n, diag), name or f"grid{n}{'w' if warp else ''}_s{seed}")


def grid_band(m: Mesh, n: int, band: int, nbands: int, halo: int = 2) -> Mesh:
    """Cell rows [band*n/nbands - halo, (band+1)*n/nbands + halo) of an n x n
    grid mesh made by jittered_grid, clipped to the grid, as a mesh of its own
    (vertices renumbered in their original order).  This is one device's share
    when a large grid is split into row bands.  On the grid, each halo row is
    one vertex ring around the band; two rings keep the repaired frontier and
    next'/prev' of every half-edge of the band proper equal to those of the
    whole mesh (a barrier tip on the outer ring can add a middle edge that
    ends on the inner one)."""
    if n % nbands or not (0 <= band < nbands) or halo < 0 or m.nt != 2 * n * n:
        raise ValueError("band of a whole n x n grid mesh, n divisible by nbands")
    rows = n // nbands
    j0 = max(0, band * rows - halo)
    j1 = min(n, (band + 1) * rows + halo)
    tri = m.tri[2 * n * j0:2 * n * j1]
    # the band's vertices are the rows j0..j1 of the (n+1)-wide vertex grid
    v0 = j0 * (n + 1)
    xy = m.xy[v0:(j1 + 1) * (n + 1)]
    return Mesh(np.ascontiguousarray(xy), np.ascontiguousarray(tri - v0),
                f"{m.name or 'grid'}_band{band}of{nbands}")


def flat_strip(n: int, name: str = "") -> Mesh:
    """2n-1 flat triangles between two horizontal lines: bases of length w on
    the lines alternate with shared sides of length sqrt(w^2/4 + h^2) < w
    (h = w/4).  Every longest edge is a boundary edge and no shared side is
    the longest edge of either triangle, so every triangle is a polygon of
    its own: P = T and Fh = 3T, the most loop half-edges a mesh can have."""
    if not (1 <= n <= 1 << 20):
        raise ValueError("n must be in [1, 2**20]")
    w = DOMAIN // n
    h = w // 4
    bot = np.stack([np.arange(n + 1, dtype=np.int64) * w, np.zeros(n + 1, np.int64)], -1)
    top = np.stack([np.arange(n, dtype=np.int64) * w + w // 2, np.full(n, h, np.int64)], -1)
    xy = np.concatenate([bot, top]).astype(np.int32)
    i = np.arange(n)
    up = np.stack([i, i + 1, n + 1 + i], -1)                  # (b_i, b_i+1, t_i)
    j = np.arange(n - 1)
    down = np.stack([n + 1 + j, j + 1, n + 2 + j], -1)       # (t_j, b_j+1, t_j+1)
    tri = np.empty((2 * n - 1, 3), np.int64)
    tri[0::2] = up
    tri[1::2] = down
    return Mesh(np.ascontiguousarray(xy), np.ascontiguousarray(tri.astype(np.int32)), name or f"flat_strip{n}")


def scrambled(m: Mesh, seed: int) -> Mesh:
    """The same triangulation numbered at random: vertices and triangles in a
    seeded random order, each triangle's corners rotated by a random shift,
    and about half of the triangles listed clockwise.  Neighbours then
    rarely share a tile, vertex ids in a tile span the whole range, and equal
    lengths are broken among scattered half-edge ids."""
    nv, nt = m.nv, m.nt
    ids = lambda lo, n: np.arange(lo, lo + n, dtype=np.uint64)
    vperm = np.argsort(uniform01(seed, _S_SCR, ids(0, nv)), kind="stable")   # new id -> old vertex
    rank = np.empty(nv, np.int64)
    rank[vperm] = np.arange(nv)
    tperm = np.argsort(uniform01(seed, _S_SCR, ids(nv, nt)), kind="stable")
    tri = rank[m.tri[tperm].astype(np.int64)]
    rot = uniform_int(seed, _S_SCR, ids(nv + nt, nt), 0, 2)
    tri = np.take_along_axis(tri, (np.arange(3)[None, :] + rot[:, None]) % 3, axis=1)
    cw = uniform_int(seed, _S_SCR, ids(nv + 2 * nt, nt), 0, 1).astype(bool)
    tri[cw] = tri[cw][:, [0, 2, 1]]
    return Mesh(np.ascontiguousarray(m.xy[vperm]), np.ascontiguousarray(tri.astype(np.int32)),
                f"{m.name}_scr{seed}")


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def plain_small() -> Mesh:
    """32 x 32 cells, jittered, random diagonals: 1,089 vertices, 2,048 triangles."""
    return jittered_grid(32, seed=0, name="plain_32x32")


def plain_scale() -> Mesh:
    """1024 x 1024 cells: 1,050,625 vertices, 2,097,152 triangles."""
    return jittered_grid(1024, seed=1, name="plain_1024x1024")


def delaunay_1m() -> Mesh:
    """Delaunay triangulation of 1M seeded random points, numbered along a
    Z-order curve: the general-position workload (1,979,675 triangles)."""
    return random_delaunay(1_000_000, 21, order="morton")


def delaunay_4m() -> Mesh:
    """Delaunay triangulation of 4M seeded random points, numbered along a
    Z-order curve: the general-position workload at the size of the paper's
    third Random mesh (Section 7.1, appendix tables; about 8M triangles).
    Qhull takes minutes for it (the points snapped onto the sides are
    collinear), so it is not part of the default benchmark run."""
    return random_delaunay(4_000_000, 21, order="morton")


def plain_large_warped() -> Mesh:
    """4096 x 4096 cells with the Gaussian-bump warp: 33,554,432 triangles."""
    return jittered_grid(4096, seed=2, warp=True, name="plain_4096x4096_warped")


def _morton(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Interleaved bits of two 21-bit coordinates (Z-order key)."""
    def spread(v):
        v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
        v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
        v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
        v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
        return v
    return spread(x) | (spread(y) << np.uint64(1))


def random_delaunay(npts: int, seed: int, snap_frac: float = 1.0 / 200, name: str = "",
                    order: str = "qhull") -> Mesh:
    """Delaunay triangulation of random integer points, after the paper's
    Random meshes (Section 7.1): points uniform in the square, points closer
    than delta = snap_frac * 2**20 to a side are moved onto that side, the four
    corners are added, duplicates are dropped.  The triangulation itself comes
    from scipy's Qhull binding (a stand-in for the Triangle code the paper
    used).  order="qhull" keeps Qhull's vertex and triangle numbering (nearly
    random in space); order="morton" renumbers both along a Z-order curve, as
    the output of a divide-and-conquer mesh generator is spatially coherent."""
    from scipy.spatial import Delaunay

    idx = np.arange(npts, dtype=np.uint64)
    x = uniform_int(seed, _S_PTS, 2 * idx, 0, DOMAIN)
    y = uniform_int(seed, _S_PTS, 2 * idx + np.uint64(1), 0, DOMAIN)
    d = int(snap_frac * DOMAIN)
    x = np.where(x < d, 0, np.where(x > DOMAIN - d, DOMAIN, x))
    y = np.where(y < d, 0, np.where(y > DOMAIN - d, DOMAIN, y))
    pts = np.concatenate([np.array([[0, 0], [DOMAIN, 0], [0, DOMAIN], [DOMAIN, DOMAIN]]),
                          np.stack([x, y], -1)])
    pts = np.unique(pts, axis=0)
    tri = Delaunay(pts).simplices
    if order == "morton":
        vkey = np.argsort(_morton(pts[:, 0], pts[:, 1]), kind="stable")
        rank = np.empty_like(vkey)
        rank[vkey] = np.arange(len(vkey))
        pts = pts[vkey]
        tri = rank[tri]
        c = pts[tri].sum(axis=1) // 3
        tri = tri[np.argsort(_morton(c[:, 0], c[:, 1]), kind="stable")]
    elif order != "qhull":
        raise ValueError(f"unknown order {order!r}")
    return Mesh(np.ascontiguousarray(pts.astype(np.int32)), np.ascontiguousarray(tri.astype(np.int32)),
                name or f"delaunay{npts}_s{seed}" + ("m" if order == "morton" else ""))


def _side_for(seed: int, stream: int, count: int, lo: float, hi: float) -> np.ndarray:
    u = uniform01(seed, stream, np.arange(count, dtype=np.uint64))
    return np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))


def batch_meshes(count: int = 512, seed: int = 3, smin: int = 16, smax: int = 512) -> list[Mesh]:
    """Independent meshes with side log-uniform in [smin, smax] cells."""
    if not (0 <= seed < 16 and count <= 1 << 16):
        raise ValueError("seed must be < 16 and count <= 65536")
    sides = np.rint(_side_for(seed, _S_MESH, count, smin, smax)).astype(int)
    out = []
    for k, s in enumerate(sides):
        sub = (seed << 16) | k
        out.append(jittered_grid(int(s), seed=sub, name=f"batch{k}_s{int(s)}"))
    return out


def served_requests(count: int, seed: int = 4, tmin: float = 1e3, tmax: float = 4e6,
                    warp_frac: float = 0.3, distinct: int = 96) -> list[Mesh]:
    """Request meshes for the served workload: triangle count log-uniform in
    [tmin, tmax] (side s = round(sqrt(T/2))), a warp_frac share warped.  To
    keep generation bounded the side is snapped to one of `distinct`
    log-spaced values and each (side, warp) mesh is generated once and shared
    by every request that draws it."""
    if not (0 <= seed < 16 and count <= 1 << 16):
        raise ValueError("seed must be < 16 and count <= 65536")
    k = np.arange(count, dtype=np.uint64)
    u_t = uniform01(seed, _S_REQ, k * np.uint64(4) + np.uint64(1))
    u_w = uniform01(seed, _S_REQ, k * np.uint64(4) + np.uint64(2))
    lo, hi = np.log(np.sqrt(tmin / 2.0)), np.log(np.sqrt(tmax / 2.0))
    side_f = np.exp(0.5 * (np.log(tmin) + u_t * (np.log(tmax) - np.log(tmin))) - 0.5 * np.log(2.0))
    grid = np.exp(np.linspace(lo, hi, distinct))
    idx = np.clip(np.rint((np.log(side_f) - lo) / (hi - lo) * (distinct - 1)).astype(int), 0, distinct - 1)
    sides = np.maximum(1, np.rint(grid[idx])).astype(int)
    warped = u_w < warp_frac
    cache: dict = {}
    out = []
    for r in range(count):
        key = (int(sides[r]), bool(warped[r]))
        if key not in cache:
            sub = (seed << 16) | (int(idx[r]) * 2 + int(warped[r]))
            cache[key] = jittered_grid(key[0], seed=sub, warp=key[1], name=f"req_s{key[0]}{'w' if key[1] else ''}")
        out.append(cache[key])
    return out


def poisson_gaps(count: int, rate_hz: float, seed: int = 4) -> np.ndarray:
    """Exponential inter-arrival gaps (seconds) of a Poisson process."""
    k = np.arange(count, dtype=np.uint64)
    u = uniform01(seed, _S_REQ, k * np.uint64(4))
    return -np.log1p(-u) / rate_hz
