// Polylla pipeline kernels for gfx950 (wave64).
//
// One run processes a batch of meshes through a per-mesh descriptor table
// (a plain call is a batch of one).  Streaming kernels tile each mesh
// separately, so a workgroup never straddles two meshes and every index it
// handles is local to one mesh; data-dependent work (barrier tips, repair
// seeds, fix-ups, loops that leave a tile) goes through small device lists
// read by persistent grids.
//
// Kernel chain (the eight kernels of the paper's Section 6 / Algorithm 7,
// regrouped so that every step reads its inputs contiguously):
//   k_label     longest edge of every triangle (Section 6.1, Algorithm 8);
//               also clears the run's counters and per-tile totals
//   k_relink    frontier bits of every half-edge (Section 6.2, Algorithm 9),
//               the seed bit of terminal edges (Section 6.3, Algorithm 10),
//               then next/prev of every frontier half-edge by turning around
//               its target / origin (Section 6.5, Algorithm 12); barrier
//               tips; every loop that closes inside the tile is walked from
//               the tile's own next' (Sections 6.5.1-6.6)
//   k_repair    middle edge at every barrier tip (Section 6.4, Algorithm 11)
//   k_fixup     next/prev again around both ends of every new frontier edge
//   k_walk      for every seed whose loop leaves its k_relink tile and every
//               seed made by the repair: walk the loop from both ends at
//               once, record its minimum and length at the minimum's
//               triangle and store it in the bucket of the minimum's
//               compaction tile (Sections 6.5.1-6.6, Algorithms 13-14)
//   k_tile_scan exclusive scan of the per-tile loop totals that k_relink and
//               k_walk accumulate (Section 6.7)
//   k_compact   writes seeds, loop offsets and the loops of every tile from
//               its prefix (Section 6.7)
//   k_emit      writes the loops no kernel stored, from both ends
//
// Label byte per triangle (tflag):
//   bits 0-1  local index of the longest edge
//   bits 2-4  frontier bit of local edges 0..2 (the repair sets more of them)
//   bit  5    the longest edge is a terminal edge and this triangle holds its
//             seed half-edge
#include "gp_internal.h"

namespace gp {

const char *const kKernelNames[K_COUNT] = {"k_label", "k_relink", "k_repair",  "k_fixup",
                                           "k_walk",  "k_tile_scan", "k_compact", "k_emit"};

constexpr uint32_t kSeedBit = 1u << 5;
constexpr uint32_t kTieBit = 1u << 7;   // written by k_label only

// The mesh arrays reached through the descriptor table live in global
// memory; saying so lets the compiler use global (not flat) loads and stores
// with a scalar base and a 32-bit offset.
#define GLOBAL __attribute__((address_space(1)))
typedef GLOBAL const int32_t *gcint;
typedef GLOBAL int32_t *gint;
typedef GLOBAL const uint8_t *gcu8;
typedef GLOBAL uint8_t *gu8;
typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v3i __attribute__((ext_vector_type(3)));
// three ints at 4-byte alignment (a v3i claims 16): loads of 12-byte records
typedef int v3i_a4 __attribute__((ext_vector_type(3), aligned(4)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef GLOBAL const v2i *gcv2i;

// ---------------------------------------------------------------------------
// half-edge queries (implicit triangle layout, Section 4.2)
// ---------------------------------------------------------------------------

// (h >= 0 everywhere these are used; unsigned division by 3 is a multiply)
__device__ __forceinline__ int tri_of(int h) { return (int)((unsigned)h / 3u); }
__device__ __forceinline__ int he_next(int h) {
    const int t = tri_of(h);
    return (h - 3 * t == 2) ? h - 2 : h + 1;
}
__device__ __forceinline__ int he_prev(int h) {
    const int t = tri_of(h);
    return (h - 3 * t == 0) ? h + 2 : h - 1;
}

__device__ __forceinline__ long long sq_len(int2 a, int2 b) {
    long long dx = (long long)b.x - a.x, dy = (long long)b.y - a.y;
    return dx * dx + dy * dy;
}

__device__ __forceinline__ bool fbit(uint32_t f, int i) { return (f >> (2 + i)) & 1u; }

__device__ __forceinline__ bool is_frontier(const uint8_t *__restrict__ tflag, int h) {
    const int t = h / 3;
    return fbit(tflag[t], h - 3 * t);
}

// Turning from candidate c (label fc of its triangle): the first frontier
// half-edge met.  NEXT: clockwise around the target of the half-edge being
// linked, c <- next(twin(c)); !NEXT: the mirror, c <- prev(twin(c)).  A
// non-frontier edge is interior, so twin(c) exists.  -1 when the guard trips.
template <bool NEXT>
__device__ __forceinline__ int turn(const int32_t *__restrict__ twin, const uint8_t *__restrict__ tflag, int c,
                                    uint32_t fc) {
    for (int k = 0; k < kRotGuard; k++) {
        const int tc = c / 3;
        if (fbit(fc, c - 3 * tc)) return c;
        const int g = twin[c];
        if (g < 0) return -1;
        c = NEXT ? he_next(g) : he_prev(g);
        fc = tflag[c / 3];
    }
    return -1;
}

__device__ __forceinline__ int turn_next(const int32_t *__restrict__ twin, const uint8_t *__restrict__ tflag,
                                         int h) {
    const int c = he_next(h);
    return turn<true>(twin, tflag, c, tflag[c / 3]);
}
__device__ __forceinline__ int turn_prev(const int32_t *__restrict__ twin, const uint8_t *__restrict__ tflag,
                                         int h) {
    const int c = he_prev(h);
    return turn<false>(twin, tflag, c, tflag[c / 3]);
}

// ---------------------------------------------------------------------------
// wave / block helpers
// ---------------------------------------------------------------------------

// v read from the lane that DPP control CTRL names, in the rows ROW_MASK
// selects; 0 where there is no such lane or the row is not selected
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_or_zero(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive scans over the 64 lanes of a wave; every lane must be active.
// Lanes form four rows of 16: shifts right by 1, 2, 4 and 8 lanes within each
// row scan the rows, then lane 15's total is added to row 1 and row 3, and
// lane 31's (rows 0-1) to rows 2 and 3.  One DPP add per step, no LDS.
__device__ __forceinline__ void wave_incl_scan2(int &a, int &b) {
    a += dpp_or_zero<0x111, 0xf>(a);   // row_shr:1
    b += dpp_or_zero<0x111, 0xf>(b);
    a += dpp_or_zero<0x112, 0xf>(a);   // row_shr:2
    b += dpp_or_zero<0x112, 0xf>(b);
    a += dpp_or_zero<0x114, 0xf>(a);   // row_shr:4
    b += dpp_or_zero<0x114, 0xf>(b);
    a += dpp_or_zero<0x118, 0xf>(a);   // row_shr:8
    b += dpp_or_zero<0x118, 0xf>(b);
    a += dpp_or_zero<0x142, 0xa>(a);   // row_bcast:15 into rows 1, 3
    b += dpp_or_zero<0x142, 0xa>(b);
    a += dpp_or_zero<0x143, 0xc>(a);   // row_bcast:31 into rows 2, 3
    b += dpp_or_zero<0x143, 0xc>(b);
}

__device__ __forceinline__ int wave_incl_scan(int a) {
    a += dpp_or_zero<0x111, 0xf>(a);
    a += dpp_or_zero<0x112, 0xf>(a);
    a += dpp_or_zero<0x114, 0xf>(a);
    a += dpp_or_zero<0x118, 0xf>(a);
    a += dpp_or_zero<0x142, 0xa>(a);
    a += dpp_or_zero<0x143, 0xc>(a);
    return a;
}

// n consecutive slots per lane from a counter, one atomic per wave (LDS or
// global memory); returns the lane's first slot.  Every lane of the wave must
// be active.
__device__ __forceinline__ int wave_alloc(int *ctr, int n) {
    const int incl = wave_incl_scan(n);
    const int tot = __builtin_amdgcn_readlane(incl, kWave - 1);
    int base = 0;
    if (tot > 0 && __lane_id() == kWave - 1) base = atomicAdd(ctr, tot);
    base = __builtin_amdgcn_readlane(base, kWave - 1);
    return base + incl - n;
}

// Exclusive block scan of a pair; lds must hold 66 ints.
__device__ __forceinline__ void block_excl_scan2(int a, int b, int &ea, int &eb, int &ta, int &tb,
                                                 int *lds) {
    int ia = a, ib = b;
    wave_incl_scan2(ia, ib);
    const int lane = __lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    if (lane == kWave - 1) {
        lds[w] = ia;
        lds[16 + w] = ib;
    }
    __syncthreads();
    if (w == 0) {
        int xa = lane < nw ? lds[lane] : 0, xb = lane < nw ? lds[16 + lane] : 0;
        int sa = xa, sb = xb;
        wave_incl_scan2(sa, sb);
        if (lane < nw) {
            lds[32 + lane] = sa - xa;
            lds[48 + lane] = sb - xb;
        }
        if (lane == nw - 1) {
            lds[64] = sa;
            lds[65] = sb;
        }
    }
    __syncthreads();
    ea = lds[32 + w] + ia - a;
    eb = lds[48 + w] + ib - b;
    ta = lds[64];
    tb = lds[65];
    __syncthreads();
}

// Mesh of a tile: the last descriptor whose first tile is <= tile.
template <int FIELD>
__device__ __forceinline__ int find_mesh(const MeshDesc *__restrict__ d, int n, int tile) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        int t0 = FIELD == 0 ? d[mid].tri_tile0 : (FIELD == 1 ? d[mid].he_tile0 : d[mid].cmp_tile0);
        if (t0 <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b on XCD b % 8)
// and each XCD has its own L2.  This gives every XCD one contiguous run of
// tiles, so the neighbour rows a tile gathers from were mostly touched by the
// same XCD.  A bijection of [0, G).
__device__ __forceinline__ int xcd_tile(int b, int G) {
    const int q = G >> 3, r = G & 7;
    const int x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Prefix sums of the stripe sizes in LDS (s_pref[0..kStripes]); returns the
// total.  Called by every thread of the block.
__device__ __forceinline__ int striped_prefix(const int32_t *counts, int cap, int *s_pref) {
    static_assert(kStripes == kWave, "one lane per stripe");
    if (threadIdx.x < kWave) {
        int c = counts[threadIdx.x * kStripePad];
        c = c < 0 ? 0 : (c > cap ? cap : c);
        int x = c;
#pragma unroll
        for (int dd = 1; dd < kWave; dd <<= 1) {
            const int y = __shfl_up(x, dd);
            if ((int)threadIdx.x >= dd) x += y;
        }
        s_pref[threadIdx.x + 1] = x;
        if (threadIdx.x == 0) s_pref[0] = 0;
    }
    __syncthreads();
    return s_pref[kStripes];
}

// Entry index of the g-th element of a striped list.
__device__ __forceinline__ int striped_index(const int *s_pref, int cap, int g) {
    int lo = 0, hi = kStripes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pref[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo * cap + (g - s_pref[lo]);
}

// Copies n ints from global src to LDS dst; src and dst 16-byte aligned.
// PER: 16-byte loads per thread that cover n (n <= 4 * PER * blockDim.x); all
// of a thread's loads are issued before the first is used.
template <int PER>
__device__ __forceinline__ void load_to_lds(int *dst, gcint src, int n) {
    const int B = blockDim.x, tid = threadIdx.x, n4 = n / 4;
    GLOBAL const v4i *s4 = reinterpret_cast<GLOBAL const v4i *>(src);
    v4i *d4 = reinterpret_cast<v4i *>(dst);
    v4i v[PER];
#pragma unroll
    for (int p = 0; p < PER; p++) {
        const int k = tid + p * B;
        v[p] = s4[k < n4 ? k : 0];
    }
#pragma unroll
    for (int p = 0; p < PER; p++) {
        const int k = tid + p * B;
        if (k < n4) d4[k] = v[p];
    }
    for (int k = (n & ~3) + tid; k < n; k += B) dst[k] = src[k];
}

// Copies n bytes from LDS src to global dst; both 4-byte aligned; every byte
// is ANDed with keep.
__device__ __forceinline__ void store_bytes_from_lds(gu8 dst, const uint8_t *src, int n, uint8_t keep) {
    const int B = blockDim.x, tid = threadIdx.x;
    const uint32_t *s4 = reinterpret_cast<const uint32_t *>(src);
    GLOBAL uint32_t *d4 = reinterpret_cast<GLOBAL uint32_t *>(dst);
    const uint32_t k4 = 0x01010101u * keep;
    for (int k = tid; k < n / 4; k += B) d4[k] = s4[k] & k4;
    for (int k = (n & ~3) + tid; k < n; k += B) dst[k] = src[k] & keep;
}

// ---------------------------------------------------------------------------
// loop records
// ---------------------------------------------------------------------------

// Loop byte of the minimum's triangle: (min(len, kPlMax) << 2) | local
// index of the minimum.  Length code 1 (no loop is that short) marks a loop
// of four whose second triangle is t + 1; its low bits then hold the local
// index of that triangle's terminal edge, and the minimum is the lower of
// the two frontier half-edges of t.
__device__ __forceinline__ uint8_t loop_code(int mn, int len) {
    return (uint8_t)(((len < kPlMax ? len : kPlMax) << 2) | (mn - 3 * tri_of(mn)));
}
constexpr int kPlQuadNext = 1;

__device__ __forceinline__ int code_len(uint32_t code) {
    const int l = (int)(code >> 2);
    return l == kPlQuadNext ? 4 : l;
}

// Where loops are stored for compaction.
struct Buckets {
    uint64_t *agg;    // per compaction tile: (loops << 32 | half-edges)
    int32_t *bcnt;    // per compaction tile: ints used
    int32_t *bucket;  // per compaction tile: cap ints
    int cap;
    int cmp_tb;       // triangles per compaction tile
};

// Stores a loop of len half-edges whose minimum mn starts it in the bucket
// of mn's compaction tile: a header, then get(0..len-1).  A bucket that
// cannot take the whole record keeps the part it has room for as a record
// nobody reads (header with local triangle 0x7fff, zeros after it), so that
// every int below the bucket's end belongs to a complete record.  Returns
// whether the loop was stored; a loop not stored is written by k_emit.
template <class GET>
__device__ __forceinline__ bool bucket_put(const Buckets &bk, const MeshDesc &d, int mn, int len, GET get) {
    const int tm = tri_of(mn), ct = tm / bk.cmp_tb;
    const size_t tile = (size_t)d.cmp_tile0 + ct;
    const int pos = atomicAdd(&bk.bcnt[tile], len + 1);
    gint rec = (gint)bk.bucket + tile * bk.cap + pos;
    if (pos + len + 1 <= bk.cap) {
        rec[0] = (int)(kRecHeader | ((uint32_t)(tm - ct * bk.cmp_tb) << 16) | (uint32_t)len);
        for (int i = 0; i < len; i++) rec[1 + i] = get(i);
        return true;
    }
    if (pos < bk.cap) {
        rec[0] = (int)(kRecHeader | (0x7fffu << 16));
        for (int i = pos + 1; i < bk.cap; i++) rec[i - pos] = 0;
    }
    return false;
}

// Adds one loop (minimum mn, length len) to the totals of mn's compaction tile.
__device__ __forceinline__ void agg_add(const Buckets &bk, const MeshDesc &d, int mn, int len) {
    atomicAdd(reinterpret_cast<unsigned long long *>(bk.agg + d.cmp_tile0 + tri_of(mn) / bk.cmp_tb),
              (1ull << 32) | (unsigned long long)(uint32_t)len);
}

// ---------------------------------------------------------------------------
// k_label: longest edge of each triangle; clears the run's counters
// ---------------------------------------------------------------------------

struct ClearArgs {
    RunCounters *rc;
    MeshCounters *ctrs;
    int nmesh;
    uint64_t *status;
    int32_t *bcnt;
    int ntiles;   // compaction tiles of the run
    int32_t *walk_counts, *emit_counts;
};

template <int ITEMS>
__global__ void __launch_bounds__(1024) k_label(const MeshDesc *__restrict__ descs, int nmesh, ClearArgs ca) {
    // the counters, list sizes and per-tile totals of the run start at zero
    // for the kernels that follow (nothing in this kernel uses them)
    {
        const int gid = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
        for (int k = gid; k < ca.ntiles; k += stride) {
            ca.status[k] = 0ull;
            ca.bcnt[k] = 0;
        }
        for (int k = gid; k < ca.nmesh; k += stride) ca.ctrs[k] = MeshCounters{};
        if (gid < kStripes) {
            ca.walk_counts[gid * kStripePad] = 0;
            ca.emit_counts[gid * kStripePad] = 0;
        }
        if (gid == 0) *ca.rc = RunCounters{};
    }
    extern __shared__ int4 lds_raw[];
    int *s_org = reinterpret_cast<int *>(lds_raw);
    const int B = blockDim.x, tid = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int mi = find_mesh<0>(descs, nmesh, tile);
    const MeshDesc &d = descs[mi];
    const int nt = d.nt;
    const int base = (tile - d.tri_tile0) * B * ITEMS;
    const gcv2i xy = (gcv2i)(d.xy);
    // the tile's corners in one contiguous load; item j of this thread is
    // triangle base + j*B + tid
    const int cnt_all = min(B * ITEMS, nt - base);
    if (cnt_all <= 0) return;   // an empty mesh's tile (the whole block)
    load_to_lds<(3 * ITEMS + 3) / 4>(s_org, (gcint)(d.org) + 3 * (size_t)base, 3 * cnt_all);
    __syncthreads();
    // every corner of every item first, so all the gathers are in flight
    // together (items past the tile read corner 0 and are dropped)
    v2i q[ITEMS][3];
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const int lt = j * B + tid;
        const int l0 = lt < cnt_all ? 3 * lt : 0;
#pragma unroll
        for (int i = 0; i < 3; i++) q[j][i] = xy[s_org[l0 + i]];
    }
    gu8 tflag = (gu8)d.tflag;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const int lt = j * B + tid;
        if (lt >= cnt_all) continue;
        const int t = base + lt;
        const int2 p0 = make_int2(q[j][0].x, q[j][0].y), p1 = make_int2(q[j][1].x, q[j][1].y),
                   p2 = make_int2(q[j][2].x, q[j][2].y);
        const long long l0 = sq_len(p0, p1), l1 = sq_len(p1, p2), l2 = sq_len(p2, p0);
        long long m = l0 > l1 ? l0 : l1;
        m = m > l2 ? m : l2;
        const int cnt = (l0 == m) + (l1 == m) + (l2 == m);
        int best = l0 == m ? 0 : (l1 == m ? 1 : 2);
        if (cnt > 1) {
            // tie at the maximum: the lower edge id min(h, twin h) wins
            best = -1;
            int bid = 0x7fffffff;
            const long long ls[3] = {l0, l1, l2};
            for (int i = 0; i < 3; i++) {
                if (ls[i] != m) continue;
                const int h = 3 * t + i, g = d.twin[h];
                const int id = (g >= 0 && g < h) ? g : h;
                if (id < bid) {
                    bid = id;
                    best = i;
                }
            }
            best |= (int)kTieBit;   // counted by k_relink
        }
        tflag[t] = (uint8_t)best;
    }
}

// ---------------------------------------------------------------------------
// k_relink: frontier and seed bits, next/prev of every frontier half-edge,
// barrier tips, loops that close inside the tile
//
// Phase 1 derives each triangle's frontier bits and seed bit from its own
// longest-edge label and its neighbours' (Section 6.2-6.3) and keeps the
// tile's label bytes and twins in LDS.  Phase 2 links every frontier
// half-edge to the next frontier half-edge around its target (next') and its
// origin (prev') (Section 6.5): the edge after it in its own triangle when
// that edge is frontier, else a turn that starts in the neighbour across it.
// The first candidate of a turn is decided by one LDS read when the
// neighbour lies in the tile; turns that go on, and candidates outside the
// tile, go to an LDS queue that the first lanes of the block run.  A
// candidate outside the tile derives its frontier bit from the longest-edge
// labels, which no kernel changes during this pass (the tile's label bytes
// are written back with their longest-edge bits unchanged).  Polygons of one
// or two triangles are settled from labels already in registers; the loops
// of other seeds are walked through the tile's next' in LDS, and those that
// leave the tile (or pass a barrier tip, which the repair will change) go to
// the walk list.
// ---------------------------------------------------------------------------

// Frontier test of half-edge c during k_relink.
struct TileLabels {
    gcint twin;
    gcu8 tflag;                          // longest-edge bits (0-1) only are read
    const int *s_tw;                     // the tile's twins
    const uint8_t *s_f;                  // the tile's label bytes, frontier bits set
    int base, cnt;                       // the tile's triangles [base, base + cnt)
};

// One step of a turn around a vertex at candidate c (Lc: the longest-edge
// label of c's triangle, or -1 when not loaded).  Returns 1 when c is a
// frontier half-edge (the turn ends there), 0 after moving c to the next
// candidate (next: c <- next(twin(c)), else c <- prev(twin(c))), -1 when the
// mesh is inconsistent.
__device__ __forceinline__ int turn_step(const TileLabels &T, int &c, int &Lc, bool next) {
    const int tc = tri_of(c), lc = c - 3 * tc, kk = tc - T.base;
    int g, Lg = -1;
    if ((unsigned)kk < (unsigned)T.cnt) {
        if (fbit(T.s_f[kk], lc)) return 1;
        g = T.s_tw[3 * kk + lc];
        if (g < 0) return -1;   // a non-frontier edge is interior
    } else {
        g = T.twin[c];
        if (g < 0) return 1;   // boundary
        if (Lc < 0) Lc = (int)(T.tflag[tc] & 3u);
        if (Lc != lc) {   // c is not its triangle's longest edge
            const int tg = tri_of(g);
            Lg = (int)(T.tflag[tg] & 3u);
            if (Lg != g - 3 * tg) return 1;   // nor is twin(c)
        }
    }
    c = next ? he_next(g) : he_prev(g);
    Lc = Lg;
    return 0;
}

// The whole turn from candidate c: the frontier half-edge it ends at, or -1.
__device__ __forceinline__ int run_turn(const TileLabels &T, int c, int Lc, bool next) {
    for (int k = 0; k < kRotGuard; k++) {
        const int r = turn_step(T, c, Lc, next);
        if (r != 0) return r > 0 ? c : -1;
    }
    return -1;
}

// Appends barrier tip he of mesh mi to the tip list.
__device__ __forceinline__ void push_tip(RunCounters *rc, ListEntry *tips, int cap_tips, const MeshDesc &d, int mi,
                                         int he, bool &err) {
    const int slot = atomicAdd(&rc->ntips, 1);
    if (slot < cap_tips) {
        tips[slot].mesh = mi;
        tips[slot].he = he;
        atomicAdd(&d.ctr->ntips, 1);
    } else {
        err = true;
    }
}

struct RelinkArgs {
    const MeshDesc *descs;
    int nmesh;
    RunCounters *rc;
    ListEntry *tips;
    int cap_tips;
    ListEntry *walk;
    int32_t *walk_counts;
    int walk_cap;
    Buckets bk;
};

// The per-block counters of k_relink in LDS.
struct RelinkShared {
    int nq;      // turns queued
    int ntip;    // tips found
    int nopen;   // seeds whose loop is walked in the tile
    int nties;
    int nwalk;   // walk-list entries of the block (reserved per wave)
    int settled_c, settled_l;   // loops settled here (block in one compaction tile)
};

template <int ITEMS>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) k_relink(RelinkArgs a) {
    extern __shared__ int4 lds_raw[];
    const int B = blockDim.x, tid = threadIdx.x, TB = B * ITEMS;
    int *s_tw = reinterpret_cast<int *>(lds_raw);                // the tile's twins
    int *s_nx = s_tw + 3 * TB;                                    // the tile's next'
    uint8_t *s_f = reinterpret_cast<uint8_t *>(s_nx + 3 * TB);   // label bytes
    uint8_t *s_pl = s_f + TB;                                     // loop bytes
    int *s_q = reinterpret_cast<int *>(s_pl + TB);                // queued turns, 2 ints each
    const int qcap = TB / 2;
    int *s_tip = s_q + 2 * qcap;                                  // barrier tips found here
    const int tcap = TB / 4;
    __shared__ RelinkShared sh;
    // loops settled here, per compaction tile, when the tile's triangles
    // span several of them (a relink tile of <= 1024 triangles, compaction
    // tiles of >= 64: at most 17)
    constexpr int kSpan = 1024 / 64 + 1;
    __shared__ int s_aggc[kSpan], s_aggl[kSpan];
    if (tid == 0) sh = RelinkShared{};
    if (tid < kSpan) {
        s_aggc[tid] = 0;
        s_aggl[tid] = 0;
    }
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int mi = find_mesh<1>(a.descs, a.nmesh, tile);
    const MeshDesc &d = a.descs[mi];
    const int nt = d.nt;
    const gcint twin = (gcint)(d.twin);
    const gu8 tflag = (gu8)(d.tflag);
    const int base = (tile - d.he_tile0) * TB;
    const int cnt = min(TB, nt - base);
    if (cnt <= 0) return;   // an empty mesh's tile (the whole block)
    const int hb = 3 * base;
    const int cmp_tb = a.bk.cmp_tb;
    // the block's triangles lie in one compaction tile unless that tile is
    // smaller than this one or not aligned with it
    const int ct0 = base / cmp_tb;
    const bool one = ct0 == (base + cnt - 1) / cmp_tb;

    // ---- phase 1: labels of the triangle and its neighbours -> frontier, seed
    // Every load is issued unconditionally (indices clamped to 0, results
    // masked after) so that all of them are in flight together.
    // per item: twins (g) and their triangles (q) as 3-vectors, so that an
    // element picked by a label is a register select, not an array in memory
    v3i g[ITEMS], q[ITEMS];
    int ties = 0;
    uint32_t f[ITEMS];    // label byte: L | frontier bits << 2 | seed bit
    uint32_t pk[ITEMS];   // bits 2i: local index of twin(3t+i); bits 6+2i: longest edge of its triangle
    {
        uint32_t own[ITEMS], fn[ITEMS][3];
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            const int lt = j * B + tid;
            const bool ok = lt < cnt;
            const v3i_a4 gv = *(GLOBAL const v3i_a4 *)(twin + 3 * (size_t)(base + (ok ? lt : 0)));
            g[j] = ok ? v3i{gv.x, gv.y, gv.z} : v3i{-1, -1, -1};
            own[j] = tflag[base + (ok ? lt : 0)];
        }
#pragma unroll
        for (int j = 0; j < ITEMS; j++)
#pragma unroll
            for (int i = 0; i < 3; i++) {
                q[j][i] = tri_of(g[j][i] < 0 ? 0 : g[j][i]);
                fn[j][i] = tflag[q[j][i]];
            }
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            const int lt = j * B + tid;
            const int t = base + lt;
            const uint32_t L = own[j] & 3u;
            ties += (lt < cnt && (own[j] & kTieBit)) ? 1 : 0;
            uint32_t out = L, p = 0;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                const int gi = g[j][i];
                const int ri = gi - 3 * q[j][i];
                const uint32_t Ln = fn[j][i] & 3u;
                const bool tl = gi >= 0 && (int)Ln == ri;   // twin is its triangle's longest edge
                // frontier: boundary, or the longest edge of neither triangle
                out |= (gi < 0 || ((int)L != i && !tl)) ? 1u << (2 + i) : 0u;
                // terminal edge: longest on both sides (the lower half-edge
                // holds the seed), or longest and on the boundary
                out |= ((int)L == i && (gi < 0 || (tl && 3 * t + i < gi))) ? kSeedBit : 0u;
                p |= ((uint32_t)(gi < 0 ? 0 : ri) << (2 * i)) | (Ln << (6 + 2 * i));
            }
            f[j] = lt < cnt ? out : 0u;
            pk[j] = p;
            if (lt < cnt) {
                s_f[lt] = (uint8_t)out;
#pragma unroll
                for (int i = 0; i < 3; i++) s_tw[3 * lt + i] = g[j][i];
            }
        }
    }
    __syncthreads();
    if (ties) atomicAdd(&sh.nties, ties);

    // ---- phase 2: first candidates, settled polygons, queued turns
    // next'/prev' of every triangle leave at once as one 12-byte store each
    // (every line written once and whole); the few turns that go on are
    // queued and their lanes patch the result in afterwards.  next' also goes
    // to LDS for the walks through the tile.
    const TileLabels T = {twin, (gcu8)tflag, s_tw, s_f, base, cnt};
    const gint nxo = (gint)(d.next_o), pvo = (gint)(d.prev_o);
    bool err = false;
    uint32_t pend[ITEMS];   // turns beyond the LDS queue: bit i next' of 3t+i, bit 3+i prev'
    int openmask = 0;       // bit j: item j holds a seed whose loop is not settled
    int scnt = 0, slen = 0; // loops settled here
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const int lt = j * B + tid;
        const int t = base + lt, h0 = 3 * t;
        const uint32_t F3 = (f[j] >> 2) & 7u;   // 0 past the tile: nothing below happens
        int cN[3], cP[3];
        uint32_t hN = 0, hP = 0;   // bit x: the first candidate across edge x is frontier
#pragma unroll
        for (int x = 0; x < 3; x++) {
            // the turns across edge x: next' of the frontier half-edge before
            // x continues at next(twin(x)), prev' of the one after x at
            // prev(twin(x)); both candidates lie in the neighbour triangle
            const int gx = g[j][x];
            const int rx = (int)((pk[j] >> (2 * x)) & 3u);
            const int rn = rx == 2 ? 0 : rx + 1, rp = rx == 0 ? 2 : rx - 1;
            cN[x] = gx - rx + rn;
            cP[x] = gx - rx + rp;
            const int k = q[j][x] - base;
            const bool in = gx >= 0 && (unsigned)k < (unsigned)cnt;
            const uint32_t fx = s_f[in ? k : 0];
            hN |= (in && ((fx >> (2 + rn)) & 1u)) ? 1u << x : 0u;
            hP |= (in && ((fx >> (2 + rp)) & 1u)) ? 1u << x : 0u;
        }
        int nv[3], pv[3];
        uint32_t pm = 0, tm = 0;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const int ia = i == 2 ? 0 : i + 1, ib = i == 0 ? 2 : i - 1;
            const bool Fi = (F3 >> i) & 1u, Fa = (F3 >> ia) & 1u, Fb = (F3 >> ib) & 1u;
            const bool hNa = (hN >> ia) & 1u, hPb = (hP >> ib) & 1u;
            nv[i] = !Fi ? -1 : (Fa ? h0 + ia : cN[ia]);
            pv[i] = !Fi ? -1 : (Fb ? h0 + ib : cP[ib]);
            pm |= (Fi && !Fa && !hNa) ? 1u << i : 0u;
            pm |= (Fi && !Fb && !hPb) ? 8u << i : 0u;
            // next'(h) == twin(h): the target of h is a barrier tip
            tm |= (Fi && !Fa && hNa && cN[ia] == g[j][i]) ? 1u << i : 0u;
        }
        if (lt < cnt) {
            *reinterpret_cast<GLOBAL v3i *>(nxo + h0) = v3i{nv[0], nv[1], nv[2]};
            *reinterpret_cast<GLOBAL v3i *>(pvo + h0) = v3i{pv[0], pv[1], pv[2]};
            // a tip half-edge's next' is kept complemented (negative) in LDS,
            // so a walk through the tile that meets it stops
#pragma unroll
            for (int i = 0; i < 3; i++) s_nx[3 * lt + i] = ((tm >> i) & 1u) ? ~nv[i] : nv[i];
        }
        // tips of this item into the tile's LDS list (rare)
        if (tm) {
#pragma unroll
            for (int i = 0; i < 3; i++) {
                if (!((tm >> i) & 1u)) continue;
                const int s = atomicAdd(&sh.ntip, 1);
                if (s < tcap)
                    s_tip[s] = 3 * lt + i;
                else
                    push_tip(a.rc, a.tips, a.cap_tips, d, mi, h0 + i, err);
            }
        }
        // A seed whose polygon is one triangle (boundary terminal edge, both
        // other edges frontier) or two (interior terminal edge, the four
        // other edges frontier) is settled here: its loop is those 3 or 4
        // half-edges.  Such polygons have no interior vertex, so no barrier
        // tip and no repair touches them.  The seed is the lower half-edge of
        // its terminal edge, so the loop's minimum lies in this triangle.
        const int L = (int)(f[j] & 3u), la = L == 2 ? 0 : L + 1, lb = L == 0 ? 2 : L - 1;
        const bool seed = (f[j] & kSeedBit) != 0;
        const bool cand = seed && ((F3 >> la) & 1u) && ((F3 >> lb) & 1u);
        const int gL = g[j][L], qL = q[j][L];
        const bool quad = ((hN & hP) >> L) & 1u;
        const int rL = (int)((pk[j] >> (2 * L)) & 3u);
        const uint32_t code = !cand ? 0u
                              : gL < 0 ? (uint32_t)loop_code(h0, 3)
                              : !quad ? 0u
                              : qL == t + 1 ? (uint32_t)((kPlQuadNext << 2) | rL)
                                            : (uint32_t)loop_code(h0 + (la < lb ? la : lb), 4);
        openmask |= (seed && !code) ? 1 << j : 0;
        if (lt < cnt) s_pl[lt] = (uint8_t)code;
        if (code) {
            if (one) {
                scnt += 1;
                slen += code_len(code);
            } else {
                const int k = t / cmp_tb - ct0;
                atomicAdd(&s_aggc[k], 1);
                atomicAdd(&s_aggl[k], code_len(code));
            }
        }
        // queue this item's open turns (one LDS atomic per wave)
        const int slot = wave_alloc(&sh.nq, __popc(pm));
        uint32_t over = 0;
        int sl = slot;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            if (!((pm >> k) & 1u)) continue;
            if (sl < qcap) {
                const int i = k % 3;
                const int x = k < 3 ? (i == 2 ? 0 : i + 1) : (i == 0 ? 2 : i - 1);
                s_q[2 * sl] = k < 3 ? cN[x] : cP[x];
                s_q[2 * sl + 1] = ((3 * lt + i) << 3) | (k < 3 ? 4 : 0) | ((int)((pk[j] >> (6 + 2 * x)) & 3u) + 1);
            } else {
                over |= 1u << k;
            }
            ++sl;
        }
        pend[j] = over;
    }
    {
        // seeds walked in the tile, and the settled totals: one LDS atomic per wave
        int o = __popc(openmask), c2 = scnt, l2 = slen;
        wave_incl_scan2(c2, l2);
        const int ot = __builtin_amdgcn_readlane(wave_incl_scan(o), kWave - 1);
        if (__lane_id() == kWave - 1) {
            if (ot) atomicAdd(&sh.nopen, ot);
            if (c2) {
                atomicAdd(&sh.settled_c, c2);
                atomicAdd(&sh.settled_l, l2);
            }
        }
    }
    __syncthreads();

    // ---- turns that go on: the queue's, spread over the block's lanes, then
    // (when the queue was full) each lane's own.  The lane that ends a turn
    // writes its result over the provisional value.
    auto finish_turn = [&](int src, bool nxt, int res) {
        err |= res < 0;
        if (nxt) {
            const bool tip = res >= 0 && res == s_tw[src];
            nxo[hb + src] = res;
            s_nx[src] = tip ? ~res : res;
            if (tip) {
                const int s = atomicAdd(&sh.ntip, 1);
                if (s < tcap)
                    s_tip[s] = src;
                else
                    push_tip(a.rc, a.tips, a.cap_tips, d, mi, hb + src, err);
            }
        } else {
            pvo[hb + src] = res;
        }
    };
    const int nq_all = sh.nq;
    const int nq = min(nq_all, qcap);
    for (int qq = tid; qq < nq; qq += B) {
        const int w = s_q[2 * qq + 1];
        finish_turn(w >> 3, (w & 4) != 0, run_turn(T, s_q[2 * qq], (w & 3) - 1, (w & 4) != 0));
    }
    if (nq_all > qcap) {   // the queue overflowed (meshes whose polygons are mostly large)
        // one loop over this lane's left-over turns, its inputs re-read from
        // LDS and the label bytes (one copy of the turn code)
        uint64_t left = 0;
#pragma unroll
        for (int j = 0; j < ITEMS; j++) left |= (uint64_t)pend[j] << (6 * j);
        while (left) {
            const int bit = __builtin_ctzll(left);
            left &= left - 1;
            const int j = bit / 6, k = bit - 6 * j, i = k % 3;
            const int lt = j * B + tid;
            const int x = k < 3 ? (i == 2 ? 0 : i + 1) : (i == 0 ? 2 : i - 1);
            const int gx = s_tw[3 * lt + x];   // interior: the turn crosses edge x
            if (gx < 0) {
                err = true;
                continue;
            }
            const int cur = k < 3 ? he_next(gx) : he_prev(gx);
            finish_turn(3 * lt + i, k < 3, run_turn(T, cur, (int)(tflag[tri_of(gx)] & 3u), k < 3));
        }
    }
    const int nopen = sh.nopen;
    if (nopen > 0) {
        if (nq_all > 0) __syncthreads();   // the patched next' in LDS
        // every seed not settled above: walk its loop through the tile
        int wlist[ITEMS];
        int npush = 0, pushm = 0;
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            wlist[j] = 0;
            if (!((openmask >> j) & 1)) continue;
            const int lt = j * B + tid;
            const int t = base + lt, h0 = 3 * t;
            const uint32_t F3 = (f[j] >> 2) & 7u;
            const int L = (int)(f[j] & 3u), la = L == 2 ? 0 : L + 1, lb = L == 0 ? 2 : L - 1;
            // a frontier half-edge of the seed's triangle lies on the loop;
            // a triangle with none starts with a search (k_walk)
            const int start = ((F3 >> la) & 1u) ? h0 + la : (((F3 >> lb) & 1u) ? h0 + lb : -1);
            if (start < 0) {
                wlist[j] = ~(h0 + L);
                pushm |= 1 << j;
                ++npush;
                continue;
            }
            int cur = start, mn = start, len = 0;
            bool closed = false;
            while (true) {
                const int idx = cur - hb;
                if ((unsigned)idx >= (unsigned)(3 * cnt)) break;   // leaves the tile
                const int nx = s_nx[idx];
                if (nx < 0) break;   // a barrier tip (or a corrupt link)
                ++len;
                mn = cur < mn ? cur : mn;
                cur = nx;
                if (cur == start) {
                    closed = true;
                    break;
                }
                if (len > 3 * cnt) break;
            }
            if (!closed) {
                wlist[j] = start;
                pushm |= 1 << j;
                ++npush;
                continue;
            }
            // the loop is settled: its byte at the minimum's triangle (in
            // this tile), its record in the bucket, its count in the totals
            s_pl[tri_of(mn) - base] = loop_code(mn, len);
            int w = mn;
            bucket_put(a.bk, d, mn, len, [&](int) {
                const int v = w;
                w = s_nx[w - hb];
                return v;
            });
            if (one) {
                atomicAdd(&sh.settled_c, 1);
                atomicAdd(&sh.settled_l, len);
            } else {
                const int k = tri_of(mn) / cmp_tb - ct0;
                atomicAdd(&s_aggc[k], 1);
                atomicAdd(&s_aggl[k], len);
            }
        }
        // loops that leave the tile: to the walk list (one atomic per wave)
        const int stripe = tile % kStripes;
        int e = wave_alloc(&a.walk_counts[stripe * kStripePad], npush);
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            if (!((pushm >> j) & 1)) continue;
            if (e < a.walk_cap) {
                a.walk[stripe * a.walk_cap + e].mesh = mi;
                a.walk[stripe * a.walk_cap + e].he = wlist[j];
            } else {
                err = true;
            }
            ++e;
        }
    }
    __syncthreads();
    // the tile's label and loop bytes in whole words (the label bytes keep
    // their longest-edge bits, which other tiles may be reading)
    store_bytes_from_lds((gu8)(d.pl) + base, s_pl, cnt, 0xff);
    store_bytes_from_lds(tflag + base, s_f, cnt, 0x3f);
    if (tid == 0) {
        if (one && sh.settled_c)
            atomicAdd(reinterpret_cast<unsigned long long *>(a.bk.agg + d.cmp_tile0 + ct0),
                      ((unsigned long long)(uint32_t)sh.settled_c << 32) | (unsigned long long)(uint32_t)sh.settled_l);
        if (sh.nties) atomicAdd(&d.ctr->nties, sh.nties);
        const int n = min(sh.ntip, tcap);   // the tile's tips: one append
        if (n > 0) {
            const int at = atomicAdd(&a.rc->ntips, n);
            atomicAdd(&d.ctr->ntips, n);
            for (int i = 0; i < n; i++) {
                if (at + i < a.cap_tips) {
                    a.tips[at + i].mesh = mi;
                    a.tips[at + i].he = hb + s_tip[i];
                } else {
                    err = true;
                }
            }
        }
    }
    if (!one && tid <= (base + cnt - 1) / cmp_tb - ct0 && s_aggc[tid] != 0)
        atomicAdd(reinterpret_cast<unsigned long long *>(a.bk.agg + d.cmp_tile0 + ct0 + tid),
                  ((unsigned long long)(uint32_t)s_aggc[tid] << 32) | (unsigned long long)(uint32_t)s_aggl[tid]);
    if (err) atomicOr(&d.ctr->err, kErrCorrupt);
}

// ---------------------------------------------------------------------------
// k_repair: middle edge of each barrier tip
// ---------------------------------------------------------------------------

// Sets the frontier bit of half-edge h; returns whether it was set before.
__device__ __forceinline__ uint32_t set_frontier_bit(uint8_t *tflag, int h) {
    int t = h / 3, i = h - 3 * t;
    uint32_t *word = reinterpret_cast<uint32_t *>(tflag) + (t >> 2);
    uint32_t bit = (1u << (2 + i)) << (8 * (t & 3));
    return atomicOr(word, bit) & bit;
}

// Appends 2 entries per lane with pred set; one atomic per wave.  Must be
// reached by every lane of the wave.
__device__ __forceinline__ int wave_reserve2(int32_t *counter, bool pred) {
    const unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return -1;
    const int lane = __lane_id(), leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, 2 * __popcll(mask));
    base = __shfl(base, leader);
    return pred ? base + 2 * __popcll(mask & ((1ull << lane) - 1ull)) : -1;
}

// The middle edge of the tip whose single frontier edge leaves it as a:
// m = CW^k(a) with k = floor(d/2), d = degree of the tip (CW(e) =
// next(twin(e))).  Two walkers leave a at once, one clockwise and one
// counter-clockwise (CCW(e) = twin(prev(e)) = CW^(d-1)(e)); after s steps
// they stand at CW^s(a) and CW^(d-s)(a), so they meet after about d/2 steps,
// and where they meet gives d and m.  -1 on a boundary or a runaway turn
// (tips are interior vertices).
__device__ __forceinline__ int middle_edge(gcint twin, int a) {
    int x = a, y = a;   // x = CW^(s-1)(a), y = CW^(d-s+1)(a)
    for (int s = 1; s <= kRotGuard / 2; s++) {
        const int gx = twin[x];                 // both loads in flight together
        const int gy = twin[he_prev(y)];
        if (gx < 0 || gy < 0) return -1;
        const int nx = he_next(gx);   // CW^s(a)
        if (nx == y) return x;        // CW^s(a) = CW^(d-s+1)(a): d = 2s - 1, m = CW^(s-1)(a)
        if (nx == gy) return nx;      // CW^s(a) = CW^(d-s)(a): d = 2s, m = CW^s(a)
        x = nx;
        y = gy;
    }
    return -1;
}

// Middle edge of every barrier tip.  Whole waves take consecutive tips, so the
// list appends and counters cost one atomic per wave (tips are many on
// general-position meshes, and atomics on one address serialize).
__global__ void k_repair(const MeshDesc *__restrict__ descs, RunCounters *rc, const ListEntry *tips,
                         int cap_tips, ListEntry *walk, int32_t *walk_counts, int walk_cap, ListEntry *fixes,
                         int cap_fix) {
    const int ntips = min(rc->ntips, cap_tips);
    const int lane = __lane_id();
    const int stride = gridDim.x * blockDim.x;
    for (int wbase = blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1)); wbase < ntips; wbase += stride) {
        const int k = wbase + lane;
        bool ok = k < ntips;
        int mesh = 0, a = -1, m = -1, mt = -1;
        bool newmid = false;
        if (ok) {
            const ListEntry e = tips[k];
            mesh = e.mesh;
            const MeshDesc &d = descs[e.mesh];
            const gcint twin = (gcint)d.twin;
            // a: the only frontier edge at the tip v = target(e.he), leaving v
            a = twin[e.he];
            m = a < 0 ? -1 : middle_edge(twin, a);
            mt = m < 0 ? -1 : twin[m];
            if (mt < 0) {
                atomicOr(&d.ctr->err, kErrCorrupt);
                ok = false;
            } else {
                newmid = !set_frontier_bit(d.tflag, m < mt ? m : mt);
                set_frontier_bit(d.tflag, m < mt ? mt : m);
            }
        }
        // both halves of the middle edge seed the polygons on either side
        const int stripe = (wbase / kWave) % kStripes;
        const int c = wave_reserve2(&walk_counts[stripe * kStripePad], ok);
        const int f = wave_reserve2(&rc->nfix, ok);
        if (ok) {
            bool full = false;
            if (c + 1 < walk_cap) {
                walk[stripe * walk_cap + c].mesh = mesh;
                walk[stripe * walk_cap + c].he = m;
                walk[stripe * walk_cap + c + 1].mesh = mesh;
                walk[stripe * walk_cap + c + 1].he = mt;
            } else {
                full = true;
            }
            if (f + 1 < cap_fix) {
                fixes[f].mesh = mesh;
                fixes[f].he = a;        // leaves the tip
                fixes[f + 1].mesh = mesh;
                fixes[f + 1].he = mt;   // leaves the other end of the middle edge
            } else {
                full = true;
            }
            if (full) atomicOr(&descs[mesh].ctr->err, kErrCorrupt);
        }
        // new middle edges, counted per mesh: one atomic per mesh in the wave
        unsigned long long pending = __ballot(ok && newmid);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int lm = __shfl(mesh, leader);
            const unsigned long long same = __ballot(ok && newmid && mesh == lm);
            if (lane == leader) atomicAdd(&descs[lm].ctr->nmiddle, __popcll(same));
            pending &= ~same;
        }
    }
}

// ---------------------------------------------------------------------------
// k_fixup: recompute next/prev of every frontier half-edge at a vertex
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool fix_around(const MeshDesc &d, int e) {
    // e leaves the vertex x; prev(e) enters x in the same triangle
    const int32_t *__restrict__ twin = d.twin;
    const uint8_t *__restrict__ tflag = d.tflag;
    const int p = he_prev(e);
    bool ok = true;
    if (is_frontier(tflag, p)) {
        const int n = turn_next(twin, tflag, p);
        ok &= n >= 0;
        d.next_o[p] = n;
    }
    if (is_frontier(tflag, e)) {
        const int q = turn_prev(twin, tflag, e);
        ok &= q >= 0;
        d.prev_o[e] = q;
    }
    return ok;
}

// Makes LDS writes of one lane visible to the other lanes of its wave.
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Every fix-up anchor o (a half-edge leaving vertex x) gets one wave.  Its
// first lane gathers the outgoing half-edges around x into LDS, walking
// clockwise and counter-clockwise from o at once (two loads in flight per
// step, about degree/2 steps), so that they lie in clockwise order.  Lane p
// then takes the p-th of them, e_p, and the half-edge entering x before it
// in the same triangle, p_p = prev(e_p).  With the frontier bits of all of
// them in two ballots, next'(p_p) is the first frontier e_j at or after p,
// and prev'(e_p) is prev of the last e_j at or before p whose p_j is
// frontier (cyclically around an interior vertex; around a boundary vertex
// both ends are boundary edges, which are frontier).  This is the turn of
// Section 6.5 for every frontier half-edge at x.  A vertex of degree above
// 62 is fixed by one lane, edge by edge.
__global__ void __launch_bounds__(256) k_fixup(const MeshDesc *__restrict__ descs, RunCounters *rc,
                                               const ListEntry *fixes, int cap_fix) {
    __shared__ int s_rot[4][2 * kWave];   // per wave: counter-clockwise list below kWave, clockwise from it
    __shared__ int s_hdr[4][4];           // per wave: first, count, closed, overflow
    const int nfix = min(rc->nfix, cap_fix);
    const int lane = __lane_id(), wv = threadIdx.x / kWave;
    int *rot = s_rot[wv];
    const int nwaves = gridDim.x * (blockDim.x / kWave);
    for (int q = blockIdx.x * (blockDim.x / kWave) + wv; q < nfix; q += nwaves) {   // wave-uniform
        const ListEntry en = fixes[q];
        const MeshDesc &d = descs[en.mesh];
        const gcint twin = (gcint)d.twin;
        const int o = en.he;
        if (lane == 0) {
            int ncw = 1, nccw = 0;
            bool closed = false, over = false, cw = true, ccw = true;
            rot[kWave] = o;
            int x = o, y = o;   // the last half-edge each walker added
            for (int s = 0; (cw || ccw) && s < kRotGuard; s++) {
                const int gx = cw ? twin[x] : 0;
                const int gy = ccw ? twin[he_prev(y)] : 0;
                cw = cw && gx >= 0;    // x has no twin: it is the clockwise-most
                ccw = ccw && gy >= 0;  // prev(y) has no twin: y is the counter-clockwise-most
                const int nx = cw ? he_next(gx) : -1;
                if (cw && nx == y) {   // around an interior vertex: every edge listed
                    closed = true;
                    break;
                }
                if (cw && ccw && nx == gy) {   // both walkers reach the same edge
                    if (ncw + nccw + 1 > kWave - 2) {
                        over = true;
                        break;
                    }
                    rot[kWave + ncw++] = nx;
                    closed = true;
                    break;
                }
                if (ncw + nccw + 2 > kWave - 2) {
                    over = cw || ccw;
                    break;
                }
                if (cw) {
                    rot[kWave + ncw++] = nx;
                    x = nx;
                }
                if (ccw) {
                    rot[kWave - 1 - nccw++] = gy;
                    y = gy;
                }
            }
            s_hdr[wv][0] = kWave - nccw;
            s_hdr[wv][1] = ncw + nccw;
            s_hdr[wv][2] = closed;
            s_hdr[wv][3] = over || (!closed && (cw || ccw));   // a runaway turn also takes the slow path
        }
        wave_sync_lds();
        const int first = s_hdr[wv][0], n = s_hdr[wv][1];
        const bool closed = s_hdr[wv][2] != 0, over = s_hdr[wv][3] != 0;
        bool ok = true;
        if (over) {
            // a vertex of very high degree: one lane turns around it, edge by
            // edge, clockwise from o and (at a boundary vertex) back the other way
            if (lane == 0) {
                int e = o;
                bool boundary = false;
                for (int s = 0; s < kRotGuard; s++) {
                    ok &= fix_around(d, e);
                    const int g = twin[e];
                    if (g < 0) {
                        boundary = true;
                        break;
                    }
                    e = he_next(g);
                    if (e == o) break;
                }
                if (boundary) {
                    e = o;
                    for (int s = 0; s < kRotGuard; s++) {
                        const int g = twin[he_prev(e)];
                        if (g < 0) break;
                        e = g;
                        ok &= fix_around(d, e);
                    }
                }
            }
        } else {
            const bool valid = lane < n;
            const int e = valid ? rot[first + lane] : 0;
            const int te = tri_of(e), le = e - 3 * te;
            const int lp = le == 0 ? 2 : le - 1;
            const uint32_t tf = valid ? ((gcu8)d.tflag)[te] : 0u;
            const bool Fe = valid && fbit(tf, le), Fp = valid && fbit(tf, lp);
            const unsigned long long mE = __ballot(Fe), mP = __ballot(Fp);
            // next'(p_p): the first frontier e_j with j >= p
            const unsigned long long ge = mE & (~0ull << lane);
            int jn = ge ? __ffsll((long long)ge) - 1 : (closed && mE ? __ffsll((long long)mE) - 1 : -1);
            // prev'(e_p): prev of the last e_j with j <= p whose p_j is frontier
            const unsigned long long le2 = mP & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
            int jp = le2 ? 63 - __clzll((long long)le2) : (closed && mP ? 63 - __clzll((long long)mP) : -1);
            const int en_ = __shfl(e, jn < 0 ? 0 : jn);
            const int ep_ = __shfl(e, jp < 0 ? 0 : jp);
            if (Fp) {
                ok &= jn >= 0;
                d.next_o[3 * te + lp] = jn >= 0 ? en_ : -1;
            }
            if (Fe) {
                ok &= jp >= 0;
                d.prev_o[e] = jp >= 0 ? he_prev(ep_) : -1;
            }
        }
        if (!ok) atomicOr(&d.ctr->err, kErrCorrupt);
        wave_sync_lds();   // the first lane overwrites the lists for the next anchor
    }
}

// ---------------------------------------------------------------------------
// k_walk: seed -> frontier half-edge -> the loop, from both ends at once
// ---------------------------------------------------------------------------

// From seed s, turn clockwise around origin(s) until a frontier half-edge.
__device__ __forceinline__ int seek_frontier(const MeshDesc &d, int s) {
    int f = s;
    for (int k = 0; k < kRotGuard; k++) {
        if (is_frontier(d.tflag, f)) return f;
        const int g = d.twin[f];
        if (g < 0) return -1;
        f = he_next(g);
    }
    return -1;
}

struct WalkArgs {
    const MeshDesc *descs;
    const ListEntry *walk;
    const int32_t *walk_counts;
    int walk_cap;
    Buckets bk;
};

// Every entry of the walk list: a frontier half-edge on a loop (or, as ~s, a
// seed s whose triangle has none: turn to one first).  Each lane walks its
// loop forward along next' and backward along prev' at once, so the two
// loads of a step are in flight together and a loop of L half-edges takes
// about L/2 steps; both ends are recorded in LDS.  When the ends meet, the
// loop's minimum and length are known: the byte at the minimum's triangle
// records them, and the loop goes to the bucket of the minimum's compaction
// tile, starting at its minimum, so k_compact places it without walking it
// again.  After a repair several seeds can walk one loop; in a mesh with
// tips every walker ORs the same byte in and only the one that found it
// empty counts and stores the loop.
__global__ void __launch_bounds__(256) k_walk(WalkArgs w) {
    __shared__ int s_pref[kStripes + 1];
    __shared__ int s_fw[kWalkBuf * 256], s_bw[kWalkBuf * 256];   // element k of lane tid at k * 256 + tid
    const int total = striped_prefix(w.walk_counts, w.walk_cap, s_pref);
    const int nthreads = gridDim.x * blockDim.x, tid = threadIdx.x;
    for (int g0 = blockIdx.x * blockDim.x; g0 < total; g0 += nthreads) {   // block-uniform
        const int gi = g0 + tid;
        int mesh = 0, start = -1;
        bool bad = false;
        if (gi < total) {
            const ListEntry e = w.walk[striped_index(s_pref, w.walk_cap, gi)];
            mesh = e.mesh;
            start = e.he >= 0 ? e.he : seek_frontier(w.descs[mesh], ~e.he);
            bad = start < 0;
        }
        const MeshDesc &d = w.descs[mesh];
        const gcint nx = (gcint)d.next_o, pv = (gcint)d.prev_o;
        const int lim = 3 * d.nt;
        int f = start, b = start, mn = start, k = 0, L = 0;
        bool act = start >= 0;
        if (act) s_fw[tid] = start;
        while (act) {
            ++k;
            const int nf = nx[f], nb = pv[b];   // both in flight together
            if (nf < 0 || nb < 0 || 2 * k > lim + 2) {
                bad = true;
                break;
            }
            if (nf == b) {   // forward reached the backward end: L = 2k - 1
                L = 2 * k - 1;
                break;
            }
            mn = nf < mn ? nf : mn;
            if (k < kWalkBuf) s_fw[k * 256 + tid] = nf;
            if (nf == nb) {   // both ends reached the same half-edge: L = 2k
                L = 2 * k;
                break;
            }
            mn = nb < mn ? nb : mn;
            if (k < kWalkBuf) s_bw[k * 256 + tid] = nb;
            f = nf;
            b = nb;
        }
        if (bad) atomicOr(&d.ctr->err, kErrCorrupt);
        if (L <= 0) continue;
        // the loop in next' order from start: nfw forward entries, then the
        // backward ones in reverse
        const int nfw = (L & 1) ? (L + 1) / 2 : L / 2 + 1;
        const bool keep = nfw <= kWalkBuf;
        auto seq = [&](int i) { return i < nfw ? s_fw[i * 256 + tid] : s_bw[(L - i) * 256 + tid]; };
        const uint32_t code = loop_code(mn, L);
        const int tm = tri_of(mn);
        bool won = true;
        if (d.ctr->ntips > 0) {
            uint32_t *wd = reinterpret_cast<uint32_t *>(d.pl) + (tm >> 2);
            const uint32_t old = atomicOr(wd, code << (8 * (tm & 3)));
            won = ((old >> (8 * (tm & 3))) & 0xffu) == 0u;
        } else {
            ((gu8)d.pl)[tm] = (uint8_t)code;   // one walker per loop without a repair
        }
        if (!won) continue;
        agg_add(w.bk, d, mn, L);
        if (keep) {
            int rot = 0;
            for (int i = 0; i < L; i++)
                if (seq(i) == mn) rot = i;
            bucket_put(w.bk, d, mn, L, [&](int i) { return seq(i + rot < L ? i + rot : i + rot - L); });
        }
    }
}

// The loops k_compact left out (no kernel stored them): each written from
// its minimum at its offset, forward along next' and backward along prev' at
// once (the length is known).
__global__ void __launch_bounds__(256) k_emit(const MeshDesc *__restrict__ descs, const EmitEntry *emit,
                                              const int32_t *emit_counts, int emit_cap) {
    __shared__ int s_pref[kStripes + 1];
    const int total = striped_prefix(emit_counts, emit_cap, s_pref);
    const int nthreads = gridDim.x * blockDim.x;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < total; g += nthreads) {
        const EmitEntry e = emit[striped_index(s_pref, emit_cap, g)];
        const MeshDesc &d = descs[e.mesh];
        const gcint nx = (gcint)d.next_o, pv = (gcint)d.prev_o;
        const gint out = (gint)d.loop_he;
        const int len = e.len, off = e.off;
        if (len <= 0 || off < 0 || off + len > 3 * d.nt) {
            atomicOr(&d.ctr->err, kErrCorrupt);
            continue;
        }
        out[off] = e.mn;
        int f = e.mn, b = e.mn;
        bool ok = true;
        const int nfw = len / 2, nbw = (len - 1) / 2;
        for (int i = 1; i <= nfw && ok; i++) {
            f = nx[f];
            int bb = b;
            if (i <= nbw) bb = pv[b];
            if (f < 0 || bb < 0) {
                ok = false;
                break;
            }
            out[off + i] = f;
            if (i <= nbw) {
                b = bb;
                out[off + len - i] = b;
            }
        }
        // the two ends must join: next' of the last forward half-edge is the
        // last backward one (or the minimum itself)
        if (!ok || nx[f] != b) atomicOr(&d.ctr->err, kErrCorrupt);
    }
}

// ---------------------------------------------------------------------------
// k_tile_scan: exclusive scan of the compaction tiles' loop totals
//
// k_relink and k_walk add every loop, once, to the total of the compaction
// tile holding its minimum: (loops << 32 | half-edges).  Per mesh, blocks of
// kScanChunk tiles turn the totals into exclusive prefixes within their
// chunk, and the last block to finish scans the chunk totals and records the
// mesh's polygon and loop half-edge counts, so each k_compact tile starts
// with its output offsets known.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(1024) k_tile_scan(const MeshDesc *__restrict__ descs, uint64_t *status,
                                                     uint64_t *cpre, int cmp_tb) {
    __shared__ int s_scan[72];
    __shared__ int s_last;
    const MeshDesc &d = descs[blockIdx.x];
    const int ntiles = d.nt > 0 ? (d.nt + cmp_tb - 1) / cmp_tb : 1;
    const int nchunks = (ntiles + kScanChunk - 1) / kScanChunk;
    const int chunk = blockIdx.y;
    if (chunk >= nchunks) return;   // the whole block
    const int tid = threadIdx.x, k = chunk * kScanChunk + tid;
    uint64_t *st = status + d.cmp_tile0;
    const uint64_t v = k < ntiles ? st[k] : 0ull;
    int ec, eh, tc, th;
    block_excl_scan2((int)(v >> 32), (int)(uint32_t)v, ec, eh, tc, th, s_scan);
    if (k < ntiles) st[k] = ((uint64_t)(uint32_t)ec << 32) | (uint32_t)eh;
    // chunk total at the chunk's first tile; the last block of the mesh turns
    // the totals into prefixes
    if (tid == 0) {
        cpre[d.cmp_tile0 + chunk * kScanChunk] = ((uint64_t)(uint32_t)tc << 32) | (uint32_t)th;
        __threadfence();
        s_last = atomicAdd(&d.ctr->chunks_done, 1) == nchunks - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    int c = 0, h = 0;
    for (int base = 0; base < nchunks; base += blockDim.x) {   // chunks beyond 1024: further rounds
        const int q = base + tid;
        uint64_t *slot = cpre + d.cmp_tile0 + (size_t)q * kScanChunk;
        const uint64_t w = q < nchunks ? __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
        int ec2, eh2, tc2, th2;
        block_excl_scan2((int)(w >> 32), (int)(uint32_t)w, ec2, eh2, tc2, th2, s_scan);
        if (q < nchunks) *slot = ((uint64_t)(uint32_t)(c + ec2) << 32) | (uint32_t)(h + eh2);
        c += tc2;
        h += th2;
    }
    if (tid == 0) {
        const bool ok = c >= 0 && h >= 0 && c <= d.nt && h <= 3 * d.nt;
        d.ctr->npoly = ok ? c : 0;
        d.ctr->nloop = ok ? h : 0;
        if (ok)
            d.loop_off[c] = h;
        else
            atomicOr(&d.ctr->err, kErrCorrupt);
    }
}

// ---------------------------------------------------------------------------
// k_compact: seeds, loop offsets and loops of every tile, from the tile's
// prefix; each tile assembles its part in LDS and writes it contiguously
// ---------------------------------------------------------------------------

// Length of the loop starting at mn (when it did not fit in the byte).
__device__ __forceinline__ int loop_length(const MeshDesc &d, int mn) {
    const gcint nx = (gcint)d.next_o;
    const int nh = 3 * d.nt;
    int cur = mn, len = 0;
    do {
        ++len;
        cur = nx[cur];
        if (cur < 0 || len > nh) return -1;
    } while (cur != mn);
    return len;
}

struct CompactArgs {
    const MeshDesc *descs;
    int nmesh;
    const uint64_t *status;
    const uint64_t *cpre;
    EmitEntry *emit;
    int32_t *emit_counts;
    int emit_cap;
    const int32_t *bcnt;
    const int32_t *bucket;
    int bucket_cap;
};

template <int ITEMS>
__global__ void __launch_bounds__(1024) k_compact(CompactArgs c) {
    extern __shared__ int4 lds_raw[];
    const int B = blockDim.x, tid = threadIdx.x;
    const int TB = B * ITEMS;
    const int he_cap = compact_he_cap(TB);
    int *s_he = reinterpret_cast<int *>(lds_raw);
    int *s_seed = s_he + he_cap;
    int *s_off = s_seed + TB;
    int *s_bk = s_off + TB;                                            // first ints of the bucket
    int16_t *s_rec = reinterpret_cast<int16_t *>(s_bk + kBucketStage);   // record of each triangle's loop
    __shared__ int s_scan[72];
    __shared__ int s_ebase;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int mi = find_mesh<2>(c.descs, c.nmesh, tile);
    const MeshDesc &d = c.descs[mi];
    const int nt = d.nt, nh = 3 * nt;
    const int ltile = tile - d.cmp_tile0;
    const int mesh_tiles = nt > 0 ? (nt + TB - 1) / TB : 1;
    const int l0 = tid * ITEMS, t0 = ltile * TB + l0;
    const gcint nx = (gcint)d.next_o;
    const gcu8 plb = (gcu8)d.pl, tfl = (gcu8)d.tflag;
    const gcint bkt = (gcint)c.bucket + (size_t)tile * c.bucket_cap;
    const int stage = min(c.bucket_cap, kBucketStage);

    // 1. everything this tile reads, issued together: its prefix, its bucket
    //    (count and first ints), and the loop and label bytes of this
    //    thread's ITEMS contiguous triangles
    const uint64_t pre = c.status[tile] + c.cpre[d.cmp_tile0 + ltile / kScanChunk * kScanChunk];
    const int pc = (int)(pre >> 32), ps = (int)(uint32_t)pre;
    const int nb = min(c.bcnt[tile], c.bucket_cap);
    constexpr int kStagePer = (kBucketStage + 63) / 64;
    int bv[kStagePer];
#pragma unroll
    for (int p = 0; p < kStagePer; p++) {
        const int k = tid + p * B;
        bv[p] = k < stage ? bkt[k] : 0;
    }
    uint8_t code[ITEMS], fl[ITEMS];
    if (ITEMS == 4 && t0 + 4 <= nt) {
        const uint32_t w = *reinterpret_cast<GLOBAL const uint32_t *>(plb + t0);
        const uint32_t v = *reinterpret_cast<GLOBAL const uint32_t *>(tfl + t0);
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            code[j] = (uint8_t)(w >> (8 * (j & 3)));
            fl[j] = (uint8_t)(v >> (8 * (j & 3)));
        }
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            code[j] = t0 + j < nt ? plb[t0 + j] : 0;
            fl[j] = t0 + j < nt ? tfl[t0 + j] : 0;
        }
    }
#pragma unroll
    for (int p = 0; p < kStagePer; p++) {
        const int k = tid + p * B;
        if (k < stage) s_bk[k] = bv[p];
    }
#pragma unroll
    for (int j = 0; j < ITEMS; j++) s_rec[l0 + j] = -1;
    __syncthreads();
    // 2. the bucket's records: each header names the local triangle of its
    //    loop's minimum
    for (int k = tid; k < nb; k += B) {
        const int v = k < stage ? s_bk[k] : bkt[k];
        if (v < 0) {
            const int lt = (v >> 16) & 0x7fff;
            if (lt < TB) s_rec[lt] = (int16_t)k;
        }
    }
    __syncthreads();
    // 3. loop lengths; the loops whose half-edges come from neither the bytes
    //    nor the bucket go to k_emit
    int lens[ITEMS], rec[ITEMS];
    bool toemit[ITEMS];
    int cnt = 0, sum = 0, nd = 0;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        lens[j] = 0;
        toemit[j] = false;
        rec[j] = s_rec[l0 + j];
        if (!code[j]) continue;
        int len = code_len(code[j]);
        if (len >= kPlMax) len = loop_length(d, 3 * (t0 + j) + (code[j] & 3));
        if (len <= 0) {
            bad = true;
            len = 0;
        }
        lens[j] = len;
        // loops of three and two-triangle loops of four are written from the
        // bytes; the rest from their bucket record, else by k_emit
        const bool quad = len == 4 && __popc((fl[j] >> 2) & 7u) == 2;
        toemit[j] = len > 0 && len != 3 && (code[j] >> 2) != kPlQuadNext && rec[j] < 0 && !quad;
        cnt += 1;
        sum += len;
        nd += toemit[j];
    }
    // 4. block scan: tile-local loop index and offset, emit-list slot
    int ecn, esum, tcn, tsum;
    block_excl_scan2(cnt | (nd << 16), sum, ecn, esum, tcn, tsum, s_scan);
    const int tcnt = tcn & 0xffff, tnd = tcn >> 16;
    const int stripe = tile % kStripes;
    if (tid == 0) {
        s_ebase = tnd > 0 ? atomicAdd(&c.emit_counts[stripe * kStripePad], tnd) : 0;
        // the tiles' prefixes must add up to the mesh totals
        if (ltile == mesh_tiles - 1 && (pc + tcnt != d.ctr->npoly || ps + tsum != d.ctr->nloop)) bad = true;
    }
    const bool fits = tsum <= he_cap && pc + tcnt <= nt && ps + tsum <= nh;
    // 5. seeds, local offsets and loops; into LDS, or straight to global
    //    memory for a tile whose loops do not fit
    // A loop of 3 is one triangle: (mn, next, prev).  A loop of 4 is two
    // triangles: the minimum's triangle has frontier half-edges a, b = next(a)
    // and crosses to the other triangle at b, whose two frontier half-edges
    // follow as p1 = next'(b), next(p1).
    __syncthreads();
    const int elim = (stripe + 1) * c.emit_cap;
    bad |= s_ebase + tnd > c.emit_cap;
    // the body is instantiated twice: loops into LDS (the tile fits, the
    // usual case), or straight to global memory; the tile decides for all
    // its threads
    auto place_loops = [&](auto he_out) {
        int q = ecn & 0xffff, off = esum, e = (ecn >> 16) + stripe * c.emit_cap + s_ebase;
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            if (!code[j]) continue;
            const int t = t0 + j;
            const uint32_t fb = (fl[j] >> 2) & 7u;
            const bool qn = (code[j] >> 2) == kPlQuadNext;
            const int mn = 3 * t + (qn ? __builtin_ctz(fb | 8u) : (code[j] & 3));
            const int len = lens[j];
            const bool place = fits || (pc + q < nt && ps + off + len <= nh);
            if (!place) {
                bad = true;
            } else {
                if (fits) {
                    s_seed[q] = mn;
                    s_off[q] = off;
                } else {
                    d.seeds[pc + q] = mn;
                    d.loop_off[pc + q] = ps + off;
                }
                if (len == 3) {
                    he_out[off] = mn;
                    he_out[off + 1] = he_next(mn);
                    he_out[off + 2] = he_prev(mn);
                } else if (qn || (len == 4 && rec[j] < 0 && !toemit[j])) {
                    // non-frontier edge sx; a = next(sx), b = prev(sx); the loop
                    // crosses sx's twin into the other triangle
                    const int sx = (fb & 1u) == 0 ? 0 : ((fb & 2u) == 0 ? 1 : 2);
                    const int aa = 3 * t + (sx == 2 ? 0 : sx + 1), bb = 3 * t + (sx == 0 ? 2 : sx - 1);
                    int p1;
                    if (qn) {   // the second triangle is t + 1: next'(b) leaves its terminal edge
                        const int Lp = code[j] & 3;
                        p1 = 3 * (t + 1) + (Lp == 2 ? 0 : Lp + 1);
                    } else {
                        p1 = nx[bb];
                    }
                    if (p1 < 0 || (mn != aa && mn != bb)) {
                        bad = true;
                    } else if (mn == aa) {
                        he_out[off] = aa;
                        he_out[off + 1] = bb;
                        he_out[off + 2] = p1;
                        he_out[off + 3] = he_next(p1);
                    } else {
                        he_out[off] = bb;
                        he_out[off + 1] = p1;
                        he_out[off + 2] = he_next(p1);
                        he_out[off + 3] = aa;
                    }
                } else if (rec[j] >= 0) {
                    // stored from its minimum by the kernel that walked it
                    const int k0 = rec[j];
                    const int hdr = k0 < stage ? s_bk[k0] : bkt[k0];
                    if ((hdr & 0xffff) != len || k0 + 1 + len > nb) {
                        bad = true;
                    } else {
                        for (int i = 0; i < len; i++) {
                            const int k = k0 + 1 + i;
                            he_out[off + i] = k < stage ? s_bk[k] : bkt[k];
                        }
                        bad |= (k0 + 1 < stage ? s_bk[k0 + 1] : bkt[k0 + 1]) != mn;
                    }
                } else {
                    if (e < elim) {
                        c.emit[e].mesh = mi;
                        c.emit[e].mn = mn;
                        c.emit[e].off = ps + off;
                        c.emit[e].len = len;
                    }
                    ++e;
                }
            }
            ++q;
            off += len;
        }
    };
    if (fits)
        place_loops(s_he);
    else
        place_loops((gint)d.loop_he + ps);
    if (fits) {
        __syncthreads();
        // contiguous stores of the tile's part of seeds, loop_off, loop_he;
        // all of a thread's LDS reads are issued before its first store
        constexpr int kSeedIt = ITEMS;                          // tcnt <= TB
        constexpr int kHeIt = (kCompactHe4 * ITEMS + 3) / 4;   // tsum <= he_cap
        const gint seeds = (gint)d.seeds, loff = (gint)d.loop_off, lhe = (gint)d.loop_he;
        int vs[kSeedIt], vo[kSeedIt], vh[kHeIt];
#pragma unroll
        for (int it = 0; it < kSeedIt; it++) {
            const int k = tid + it * B;
            vs[it] = s_seed[k < tcnt ? k : 0];
            vo[it] = s_off[k < tcnt ? k : 0];
        }
#pragma unroll
        for (int it = 0; it < kHeIt; it++) {
            const int k = tid + it * B;
            vh[it] = s_he[k < tsum ? k : 0];
        }
#pragma unroll
        for (int it = 0; it < kSeedIt; it++) {
            const int k = tid + it * B;
            if (k < tcnt) {
                seeds[pc + k] = vs[it];
                loff[pc + k] = ps + vo[it];
            }
        }
#pragma unroll
        for (int it = 0; it < kHeIt; it++) {
            const int k = tid + it * B;
            if (k < tsum) lhe[ps + k] = vh[it];
        }
    }
    if (bad) atomicOr(&d.ctr->err, kErrCorrupt);
}

// ---------------------------------------------------------------------------
// small copies between device memory and coherent pinned host memory (the
// descriptor table before a run, the per-mesh counters after it): a kernel
// in stream order instead of the runtime's copy path
// ---------------------------------------------------------------------------

__global__ void k_copy_words(uint32_t *dst, const uint32_t *src, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

hipError_t launch_copy_words(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (bytes % 4 || bytes / 4 > 0x7fffffff) return hipErrorInvalidValue;
    const int n = (int)(bytes / 4);
    if (n == 0) return hipSuccess;
    const int grid = (n + 255) / 256 < 64 ? (n + 255) / 256 : 64;
    hipLaunchKernelGGL(k_copy_words, dim3(grid), dim3(256), 0, s, static_cast<uint32_t *>(dst),
                       static_cast<const uint32_t *>(src), n);
    return hipGetLastError();
}

__global__ void k_put_desc(MeshDesc d, MeshDesc *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = d;
}

hipError_t launch_put_desc(const MeshDesc &d, MeshDesc *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, d, dst);
    return hipGetLastError();
}

__global__ void k_export_counts(const MeshCounters *c, int32_t *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const MeshCounters k = *c;
        out[0] = k.err ? -10 : 0;   // GP_ECORRUPT
        out[1] = k.npoly;
        out[2] = k.nloop;
        out[3] = k.ntips;
        out[4] = k.nmiddle;
        out[5] = k.nties;
        out[6] = 0;
        out[7] = 0;
    }
}

hipError_t launch_export_counts(const MeshCounters *c, int32_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_export_counts, dim3(1), dim3(64), 0, s, c, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// host launch of the whole chain
// ---------------------------------------------------------------------------

#define GP_LAUNCH_ITEMS(KER, ITEMS_RT, GRID, BLOCK, LDS, STREAM, ...)                            \
    do {                                                                                      \
        switch (ITEMS_RT) {                                                                   \
            case 1: hipLaunchKernelGGL(KER<1>, GRID, BLOCK, LDS, STREAM, __VA_ARGS__); break; \
            case 2: hipLaunchKernelGGL(KER<2>, GRID, BLOCK, LDS, STREAM, __VA_ARGS__); break; \
            case 4: hipLaunchKernelGGL(KER<4>, GRID, BLOCK, LDS, STREAM, __VA_ARGS__); break; \
            case 8: hipLaunchKernelGGL(KER<8>, GRID, BLOCK, LDS, STREAM, __VA_ARGS__); break; \
            default: return hipErrorInvalidValue;                                             \
        }                                                                                     \
    } while (0)

hipError_t launch_pipeline(const LaunchCfg &cfg, const RunBuffers &rb, hipStream_t s, launch_hook hook,
                           void *user) {
    auto H = [&](int k, int after) {
        if (hook) hook(user, k, after);
    };
    if (rb.nmesh <= 0) return hipSuccess;
    const int pb = cfg.persistent_blocks, pt = cfg.block_persistent;
    const int cmp_tb = cfg.block_compact * cfg.items_compact;   // triangles per compaction tile
    const Buckets bk = {rb.status, rb.bcnt, rb.bucket, rb.bucket_cap, cmp_tb};

    H(K_LABEL, 0);
    {
        const ClearArgs ca = {rb.rc, rb.ctrs, rb.nmesh, rb.status, rb.bcnt, rb.cmp_tiles, rb.walk_counts,
                              rb.emit_counts};
        GP_LAUNCH_ITEMS(k_label, cfg.items_label, dim3(rb.tri_tiles), dim3(cfg.block_label),
                        sizeof(int) * 3 * (size_t)cfg.block_label * cfg.items_label, s, rb.descs, rb.nmesh, ca);
    }
    H(K_LABEL, 1);

    H(K_RELINK, 0);
    {
        const RelinkArgs ra = {rb.descs, rb.nmesh, rb.rc, rb.tips, rb.cap_tips, rb.walk, rb.walk_counts,
                               rb.walk_cap, bk};
        GP_LAUNCH_ITEMS(k_relink, cfg.items_relink, dim3(rb.he_tiles), dim3(cfg.block_relink),
                        (sizeof(int) * 6 + 2 + 4 + 1) * (size_t)cfg.block_relink * cfg.items_relink, s, ra);
    }
    H(K_RELINK, 1);

    H(K_REPAIR, 0);
    hipLaunchKernelGGL(k_repair, dim3(pb), dim3(pt), 0, s, rb.descs, rb.rc, rb.tips, rb.cap_tips, rb.walk,
                       rb.walk_counts, rb.walk_cap, rb.fixes, rb.cap_fix);
    H(K_REPAIR, 1);

    H(K_FIXUP, 0);
    hipLaunchKernelGGL(k_fixup, dim3(pb), dim3(256), 0, s, rb.descs, rb.rc, rb.fixes, rb.cap_fix);
    H(K_FIXUP, 1);

    H(K_WALK, 0);
    {
        const WalkArgs wa = {rb.descs, rb.walk, rb.walk_counts, rb.walk_cap, bk};
        hipLaunchKernelGGL(k_walk, dim3(pb), dim3(256), 0, s, wa);
    }
    H(K_WALK, 1);

    H(K_TSCAN, 0);
    hipLaunchKernelGGL(k_tile_scan, dim3(rb.nmesh, rb.max_chunks), dim3(1024), 0, s, rb.descs, rb.status,
                       rb.cpre, cmp_tb);
    H(K_TSCAN, 1);

    H(K_COMPACT, 0);
    {
        const CompactArgs ca = {rb.descs, rb.nmesh,        rb.status, rb.cpre,   rb.emit,
                                rb.emit_counts, rb.emit_cap, rb.bcnt,   rb.bucket, rb.bucket_cap};
        GP_LAUNCH_ITEMS(k_compact, cfg.items_compact, dim3(rb.cmp_tiles), dim3(cfg.block_compact),
                        compact_lds_bytes(cmp_tb), s, ca);
    }
    H(K_COMPACT, 1);

    H(K_EMIT, 0);
    hipLaunchKernelGGL(k_emit, dim3(pb), dim3(256), 0, s, rb.descs, rb.emit, rb.emit_counts, rb.emit_cap);
    H(K_EMIT, 1);
    return hipGetLastError();
}

}  // namespace gp
