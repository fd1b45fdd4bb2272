// Polylla pipeline kernels for gfx950 (wave64).
//
// One run processes a batch of meshes through a per-mesh descriptor table
// (a plain call is a batch of one).  Streaming kernels tile each mesh
// separately, so a workgroup never straddles two meshes and every index it
// handles is local to one mesh; data-dependent work (barrier tips, repair
// seeds, fix-ups) goes through small device lists read by persistent grids.
//
// Kernel chain (the eight kernels of the paper's Section 6 / Algorithm 7,
// regrouped so that every step reads its inputs contiguously):
//   k_label     longest edge of every triangle (Section 6.1, Algorithm 8);
//               also clears the run's counters and per-tile totals
//   k_relink    frontier bits of every half-edge (Section 6.2, Algorithm 9),
//               the seed bit of terminal edges (Section 6.3, Algorithm 10),
//               then next/prev of every frontier half-edge by turning around
//               its target / origin (Section 6.5, Algorithm 12); barrier tips
//   k_repair    middle edge at every barrier tip (Section 6.4, Algorithm 11)
//   k_fixup     next/prev again around both ends of every new frontier edge
//   k_walk      for every seed k_relink left open and every seed made by the
//               repair: move to a frontier half-edge of its polygon
//               (Section 6.5.1, Algorithm 13), walk the loop, and record its
//               minimum and length at the minimum's triangle (Section 6.6,
//               Algorithm 14).  Polygons of one or two triangles are settled
//               by k_relink itself.
//   k_tile_scan exclusive scan of the per-tile loop totals that k_relink and
//               k_walk accumulate (Section 6.7)
//   k_compact   writes seeds, loop offsets and the loops of up to four
//               half-edges of every tile from its prefix (Section 6.7)
//   k_emit      writes the longer loops at the offsets k_compact reserved
//
// Label byte per triangle (tflag):
//   bits 0-1  local index of the longest edge
//   bits 2-4  frontier bit of local edges 0..2 (the repair sets more of them)
//   bit  5    the longest edge is a terminal edge and this triangle holds its
//             seed half-edge
//   bit  6    k_walk stored the loop whose minimum lies in this triangle
//   bit  7    (from k_label to k_relink only) the longest edge is tied
#include "gp_internal.h"

namespace gp {

const char *const kKernelNames[K_COUNT] = {"k_label",     "k_relink",  "k_repair", "k_fixup",
                                           "k_walk", "k_tile_scan", "k_compact", "k_emit", "k_small"};

constexpr uint32_t kSeedBit = 1u << 5;

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

// Value of escaped field key of a compact mesh (the table holds every key an
// escaped field can ask for; -1 for an absent key: a corrupt table).
__device__ __forceinline__ int esc_lookup(const int32_t *__restrict__ esc, int32_t mask, int32_t key) {
    uint32_t slot = esc_hash(key) & (uint32_t)mask;
    for (int k = 0; k <= mask; k++) {
        const int32_t kk = esc[2 * slot];
        if (kk == key) return esc[2 * slot + 1];
        if (kk == kEscEmpty) break;
        slot = (slot + 1) & (uint32_t)mask;
    }
    return -1;
}

// Twins of a mesh, in either encoding: twin[h] (-1 on the boundary).  The
// encoding is the same for every lane of a launch over one mesh, so the
// branch on it is uniform.
struct TwinView {
    GLOBAL const int32_t *t32;
    GLOBAL const int16_t *t16;   // compact: twin - h (0: boundary, kEsc16: escaped)
    const int32_t *esc;
    int32_t mask;
    __device__ __forceinline__ int operator[](int h) const {
        if (!t16) return t32[h];
        const int v = t16[h];
        if (v == 0) return -1;
        return v != kEsc16 ? h + v : esc_lookup(esc, mask, h);
    }
};

__device__ __forceinline__ TwinView twin_view(const MeshDesc &d) {
    return TwinView{(GLOBAL const int32_t *)d.twin, (GLOBAL const int16_t *)d.twin16, d.esc, d.esc_mask};
}
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

// Coordinates lie in [0, 2^30] (the build checks them), so a difference fits
// 32 bits and each square is one signed 32 x 32 -> 64-bit multiply.
__device__ __forceinline__ long long sq_len(int2 a, int2 b) {
    const int dx = b.x - a.x, dy = b.y - a.y;
    return (long long)dx * dx + (long long)dy * dy;
}

__device__ __forceinline__ bool fbit(uint32_t f, int i) { return (f >> (2 + i)) & 1u; }

__device__ __forceinline__ bool is_frontier(const uint8_t *__restrict__ tflag, int h) {
    const int t = h / 3;
    return fbit(tflag[t], h - 3 * t);
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

// ---------------------------------------------------------------------------
// k_label: longest edge of each triangle
// ---------------------------------------------------------------------------

// What a run clears before its kernels count into it.
struct ClearArgs {
    RunCounters *rc;
    MeshCounters *ctrs;
    uint64_t *status;   // per compaction tile
    int nstatus;
    int32_t *walk_counts, *emit_counts, *wbuf_counts;
};

// Label byte bit 7: the maximum edge length of the triangle is tied (k_label
// sets it, k_relink counts it and writes the byte back without it).
constexpr uint32_t kTieBit = 1u << 7;

template <int ITEMS>
__global__ void __launch_bounds__(1024) k_label(const MeshDesc *__restrict__ descs, int nmesh, ClearArgs ca) {
    // the run's counters, list sizes and per-tile totals start at zero for
    // the kernels that follow (nothing in this kernel counts into them)
    {
        const int gid = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
        for (int k = gid; k < ca.nstatus; k += stride) ca.status[k] = 0ull;
        for (int k = gid; k < nmesh; k += stride) ca.ctrs[k] = MeshCounters{};
        if (gid < kStripes) {
            ca.walk_counts[gid * kStripePad] = 0;
            ca.emit_counts[gid * kStripePad] = 0;
            ca.wbuf_counts[gid * kStripePad] = 0;
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
    if (!d.org8) {   // (uniform)
        load_to_lds<(3 * ITEMS + 3) / 4>(s_org, (gcint)(d.org) + 3 * (size_t)base, 3 * cnt_all);
    } else {   // a compact mesh: v0 and two 16-bit offsets per triangle
        GLOBAL const v2i *o8 = (GLOBAL const v2i *)d.org8 + base;
        for (int k = tid; k < cnt_all; k += B) {
            const v2i r = o8[k];
            const int d1 = (int)(int16_t)(r.y & 0xffff), d2 = r.y >> 16;
            const int h = 3 * (base + k);
            s_org[3 * k] = r.x;
            s_org[3 * k + 1] = d1 != kEsc16 ? r.x + d1 : esc_lookup(d.esc, d.esc_mask, ~(h + 1));
            s_org[3 * k + 2] = d2 != kEsc16 ? r.x + d2 : esc_lookup(d.esc, d.esc_mask, ~(h + 2));
        }
    }
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
                const int h = 3 * t + i, g = twin_view(d)[h];
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
// barrier tips
//
// One thread per triangle.  Phase 1 derives each triangle's frontier bits
// and seed bit from its own longest-edge label and its neighbours' (Section
// 6.2-6.3) and keeps the byte in LDS.  Phase 2 turns around the ends of every
// frontier half-edge (Section 6.5): a candidate in the tile reads its
// frontier bit from LDS; one outside derives it from the longest-edge labels,
// which no kernel changes during this pass (the tile's label bytes are
// written back with their longest-edge bits unchanged).  Each thread loads
// its triangles' twins and stores their next'/prev' itself (12 contiguous
// bytes per triangle); the label and loop bytes go out through LDS in whole
// words.
// ---------------------------------------------------------------------------

// Loop byte of the minimum's triangle: (min(len, kPlMax) << 2) | local
// index of the minimum.  Length code 1 (no loop is that short) marks a loop
// of four whose second triangle is t + 1; its low bits then hold the local
// index of that triangle's terminal edge, and the minimum is the lower of
// the two frontier half-edges of t.
__device__ __forceinline__ uint8_t loop_code(int mn, int len) {
    return (uint8_t)(((len < kPlMax ? len : kPlMax) << 2) | (mn % 3));
}
constexpr int kPlQuadNext = 1;

// Records a walked loop (minimum mn, length len) once: the walker that sets
// the byte of the minimum's triangle adds the loop to the totals of that
// triangle's compaction tile.  After a repair several seeds of one polygon
// walk the same loop; only the first counts it.  claim_issue ORs the code in
// and returns the word as it was (every walker of the loop writes the same
// code, so OR-ing is safe); claim_won reads the verdict from it, so other
// memory operations can be issued while the atomic is in flight.
__device__ __forceinline__ uint32_t claim_issue(const MeshDesc &d, int mn, int len) {
    const int tm = tri_of(mn);
    uint32_t *w = reinterpret_cast<uint32_t *>(d.pl) + (tm >> 2);
    return atomicOr(w, (uint32_t)loop_code(mn, len) << (8 * (tm & 3)));
}
__device__ __forceinline__ bool claim_won(const MeshDesc &d, uint32_t old, int mn, int len, uint64_t *agg,
                                          int cmp_tb) {
    const int tm = tri_of(mn);
    if ((old >> (8 * (tm & 3))) & 0xffu) return false;
    atomicAdd(reinterpret_cast<unsigned long long *>(agg + d.cmp_tile0 + tm / cmp_tb),
              (1ull << 32) | (unsigned long long)(uint32_t)len);
    return true;
}

// Label bit 6 of a loop's minimum triangle: k_walk stored the loop in the
// scratch pool (at lpos of that triangle); k_relink writes the label bytes
// with the bit clear.
constexpr uint32_t kStoredBit = 1u << 6;

// Copies n bytes from LDS src to global dst; both 4-byte aligned.
__device__ __forceinline__ void store_bytes_from_lds(gu8 dst, const uint8_t *src, int n) {
    const int B = blockDim.x, tid = threadIdx.x;
    const uint32_t *s4 = reinterpret_cast<const uint32_t *>(src);
    GLOBAL uint32_t *d4 = reinterpret_cast<GLOBAL uint32_t *>(dst);
    for (int k = tid; k < n / 4; k += B) d4[k] = s4[k];
    for (int k = (n & ~3) + tid; k < n; k += B) dst[k] = src[k];
}

// Frontier test of half-edge c during k_relink.  Lc is the longest-edge label
// of c's triangle, or -1 when it has not been loaded.
struct TileLabels {
    TwinView twin;
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
        const uint32_t fc = Lc < 0 ? T.tflag[tc] : 0u;   // in flight with the twin
        if (g < 0) return 1;   // boundary
        if (Lc < 0) Lc = (int)(fc & 3u);
        if (Lc != lc) {   // c is not its triangle's longest edge
            // twin(c)'s triangle is often back in the tile, whose label
            // bytes (longest-edge bits unchanged) are in LDS
            const int tg = tri_of(g), kg = tg - T.base;
            Lg = (int)(((unsigned)kg < (unsigned)T.cnt ? (uint32_t)T.s_f[kg] : (uint32_t)T.tflag[tg]) & 3u);
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

// Records a barrier tip found in a k_relink tile in the tile's LDS list
// (appended to the global list once per block); straight to the global list
// when the LDS list is full.
__device__ __forceinline__ void tile_tip(int *s_tip, int *s_ntip, int tcap, int local_he, int base, RunCounters *rc,
                                         ListEntry *tips, int cap_tips, const MeshDesc &d, int mi, bool &err);

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

__device__ __forceinline__ void tile_tip(int *s_tip, int *s_ntip, int tcap, int local_he, int base, RunCounters *rc,
                                         ListEntry *tips, int cap_tips, const MeshDesc &d, int mi, bool &err) {
    const int i = atomicAdd(s_ntip, 1);
    if (i < tcap)
        s_tip[i] = local_he;
    else
        push_tip(rc, tips, cap_tips, d, mi, 3 * base + local_he, err);
}

// Frontier bit of half-edge c of a triangle outside the tile whose
// longest-edge label is Lc.
__device__ __forceinline__ bool outside_fbit(const TileLabels &T, int c, int Lc) {
    const int tc = c / 3, lc = c - 3 * tc;
    if (Lc == lc) return false;
    const int g = T.twin[c];
    if (g < 0) return true;
    const int tg = g / 3;
    return (int)(T.tflag[tg] & 3u) != g - 3 * tg;
}

// CM: some mesh of the run is compact (else the int32 twins are read
// without a test of the encoding).  NT: next'/prev' go out as streaming
// (nontemporal) stores.
template <int ITEMS, bool CM, bool NT>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) k_relink(const MeshDesc *__restrict__ descs, int nmesh,
                                                  RunCounters *rc, ListEntry *tips, int cap_tips,
                                                  ListEntry *walk, int32_t *walk_counts, int walk_cap,
                                                  uint64_t *agg, int cmp_tb) {
    extern __shared__ int4 lds_raw[];
    int *lds = reinterpret_cast<int *>(lds_raw);
    const int B = blockDim.x, tid = threadIdx.x, TB = B * ITEMS;
    int *s_tw = lds;                                            // the tile's twins
    uint8_t *s_f = reinterpret_cast<uint8_t *>(lds + 3 * TB);   // label bytes
    uint8_t *s_pl = s_f + TB;                                   // loop bytes
    int *s_q = reinterpret_cast<int *>(s_pl + TB);              // queued turns, 2 ints each
    const int qcap = TB / 2;
    int *s_tip = s_q + 2 * qcap;                                // barrier tips found here
    const int tcap = TB / 4;
    __shared__ int s_ntip;
    // loops settled here, per compaction tile, when the tile's triangles
    // span several of them (a relink tile of <= 1024 triangles, compaction
    // tiles of >= 64: at most 17)
    constexpr int kSpan = 1024 / 64 + 1;
    __shared__ int s_aggc[kSpan], s_aggl[kSpan];
    if (threadIdx.x == 0) s_ntip = 0;
    if (threadIdx.x < kSpan) {
        s_aggc[threadIdx.x] = 0;
        s_aggl[threadIdx.x] = 0;
    }
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int mi = find_mesh<1>(descs, nmesh, tile);
    const MeshDesc &d = descs[mi];
    const int nt = d.nt;
    TwinView twin = twin_view(d);
    if (!CM) twin.t16 = nullptr;
    const gu8 tflag = (gu8)(d.tflag);
    const gint nxo = (gint)(d.next_o), pvo = (gint)(d.prev_o);
    const int base = (tile - d.he_tile0) * TB;
    const int cnt = min(TB, nt - base);
    if (cnt <= 0) return;   // an empty mesh's tile (the whole block)
    // phase 1: labels of the triangle and its neighbours -> frontier, seed.
    // Each thread loads its triangles' twins itself (12 contiguous bytes per
    // triangle, so a wave's loads are contiguous) and issues the label
    // gathers as soon as they arrive; the twins go to LDS for the turns of
    // phase 2, published by the barrier after the label bytes.  Every load is
    // issued unconditionally (indices clamped to 0, results masked after) so
    // that all of them are in flight together.
    int tw[ITEMS][3];
    uint32_t f[ITEMS], fn[ITEMS][3];
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const int lt = j * B + tid;
        const bool ok = lt < cnt;
        const int hj = 3 * (base + (ok ? lt : 0));
        v3i_a4 g;
        if (!twin.t16) {   // (uniform) one 12-byte load
            g = *(GLOBAL const v3i_a4 *)(twin.t32 + hj);
        } else {
            g.x = twin[hj];
            g.y = twin[hj + 1];
            g.z = twin[hj + 2];
        }
        tw[j][0] = ok ? g.x : -1;
        tw[j][1] = ok ? g.y : -1;
        tw[j][2] = ok ? g.z : -1;
        f[j] = tflag[base + (ok ? lt : 0)];
#pragma unroll
        for (int i = 0; i < 3; i++) fn[j][i] = tflag[tri_of(tw[j][i] < 0 ? 0 : tw[j][i])];
    }
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const int lt = j * B + tid;
        if (lt < cnt) {
#pragma unroll
            for (int i = 0; i < 3; i++) s_tw[3 * lt + i] = tw[j][i];
        }
    }
    int ties = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const int lt = j * B + tid;
        const int t = base + lt;
        const uint32_t L = f[j] & 3u;
        ties += (lt < cnt && (f[j] & kTieBit)) ? 1 : 0;
        uint32_t out = L;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const int g = tw[j][i];
            fn[j][i] = g >= 0 ? fn[j][i] & 3u : 0u;
            const bool twin_long = g >= 0 && (int)fn[j][i] == g - 3 * tri_of(g);
            // frontier: boundary, or the longest edge of neither triangle
            out |= (g < 0 || ((int)L != i && !twin_long)) ? 1u << (2 + i) : 0u;
            // terminal edge: longest on both sides (the lower half-edge holds
            // the seed), or longest and on the boundary
            out |= ((int)L == i && (g < 0 || (twin_long && 3 * t + i < g))) ? kSeedBit : 0u;
        }
        f[j] = lt < cnt ? out : 0u;
        if (lt < cnt) s_f[lt] = (uint8_t)out;
    }
    if (ties) atomicAdd(&d.ctr->nties, ties);   // (rare)
    __syncthreads();
    // phase 2: next'/prev' of every frontier half-edge.  The next (previous)
    // edge in the triangle is taken when it is frontier itself; otherwise the
    // turn continues in the neighbour across it.  A triangle has at most one
    // frontier half-edge followed by a non-frontier one and at most one
    // preceded by one, so each item has at most two turns; nearly all of
    // them end at their first candidate.  The common path is straight-line
    // code; only turns that go on, and candidates outside the tile, branch.
    const TileLabels T = {twin, tflag, s_tw, s_f, base, cnt};
    bool err = false;
    int openmask = 0;   // bit j: item j holds a seed whose loop k_walk must walk
    int scnt = 0, slen = 0;   // loops settled here: count, half-edges
    uint8_t codes[ITEMS];
    uint32_t pend = 0;  // bit 2j (2j+1): the next' (prev') turn of item j goes on
    int cur[2 * ITEMS], lab[2 * ITEMS], src[2 * ITEMS];   // turn state; src: the
                                                          // local index of the half-edge
    int nv3[ITEMS][3], pv3[ITEMS][3];                     // this lane's next'/prev'
    int qslot[2 * ITEMS];                                 // LDS queue slot of turn k, or -1
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const int lt = j * B + tid;   // lt >= cnt: f[j] == 0, so nothing is queued
        const int h0 = 3 * (base + lt);
        const uint32_t F3 = (f[j] >> 2) & 7u;
        const uint32_t rn = ((F3 >> 1) | (F3 << 2)) & 7u;   // bit i: edge i+1 frontier
        const uint32_t rp = ((F3 << 1) | (F3 >> 2)) & 7u;   // bit i: edge i-1 frontier
        const uint32_t mn = F3 & ~rn, mp = F3 & ~rp;        // at most one bit each
        // in-triangle values (the turn's slot gets its value when the turn ends)
        int nxv[3], pvv[3];
#pragma unroll
        for (int i = 0; i < 3; i++) {
            nxv[i] = ((F3 & rn) >> i) & 1u ? h0 + (i == 2 ? 0 : i + 1) : -1;
            pvv[i] = ((F3 & rp) >> i) & 1u ? h0 + (i == 0 ? 2 : i - 1) : -1;
        }
        // next' turn: from the frontier half-edge na, across x = next(na)
        const int na = mn ? __builtin_ctz(mn) : 0, x = na == 2 ? 0 : na + 1;
        const int ux = x == 0 ? tw[j][0] : (x == 1 ? tw[j][1] : tw[j][2]);
        src[2 * j] = 3 * lt + na;
        cur[2 * j] = he_next(ux < 0 ? 0 : ux);
        lab[2 * j] = (int)(x == 0 ? fn[j][0] : (x == 1 ? fn[j][1] : fn[j][2]));
        // prev' turn: from the frontier half-edge pa, across y = prev(pa)
        const int pa = mp ? __builtin_ctz(mp) : 0, y = pa == 0 ? 2 : pa - 1;
        const int uy = y == 0 ? tw[j][0] : (y == 1 ? tw[j][1] : tw[j][2]);
        src[2 * j + 1] = 3 * lt + pa;
        cur[2 * j + 1] = he_prev(uy < 0 ? 0 : uy);
        lab[2 * j + 1] = (int)(y == 0 ? fn[j][0] : (y == 1 ? fn[j][1] : fn[j][2]));
        // a non-frontier edge is interior: ux, uy >= 0 whenever the turn exists
        err |= (mn && ux < 0) || (mp && uy < 0);
        // first candidates: most are frontier half-edges of a triangle in the
        // tile, which ends the turn at once
        const int cn = cur[2 * j], tn = tri_of(cn), kn = tn - base;
        const int cp = cur[2 * j + 1], tq = tri_of(cp), kq = tq - base;
        const bool inn = (unsigned)kn < (unsigned)cnt, inq = (unsigned)kq < (unsigned)cnt;
        const uint32_t fbn = s_f[inn ? kn : 0], fbq = s_f[inq ? kq : 0];
        const bool hitn = mn && inn && fbit(fbn, cn - 3 * tn);
        const bool hitq = mp && inq && fbit(fbq, cp - 3 * tq);
        if (hitn) {
            // next'(h) == twin(h): the target of h is a barrier tip
            if (cn == (na == 0 ? tw[j][0] : (na == 1 ? tw[j][1] : tw[j][2])))
                tile_tip(s_tip, &s_ntip, tcap, 3 * lt + na, base, rc, tips, cap_tips, d, mi, err);
        }
        const bool pn = mn && !hitn, pp = mp && !hitq;   // turns that go on
        pend |= (pn ? 1u : 0u) << (2 * j) | (pp ? 1u : 0u) << (2 * j + 1);
        // this triangle's next'/prev' stay in registers until the tile is done
        // (a turn that goes on fills its slot later), then go out as one
        // 12-byte store each, so every line is written once and whole
#pragma unroll
        for (int i = 0; i < 3; i++) {
            nv3[j][i] = (mn && i == na) ? cn : nxv[i];
            pv3[j][i] = (mp && i == pa) ? cp : pvv[i];
        }
    }
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const int lt = j * B + tid;
        const int t = base + lt, h0 = 3 * t;
        // A seed whose polygon is one triangle (boundary terminal edge, both
        // other edges frontier) or two (interior terminal edge, the four
        // other edges frontier) is settled here: its loop is those 3 or 4
        // half-edges.  Such polygons have no interior vertex, so no barrier
        // tip and no repair touches them.  The seed is the lower half-edge of
        // its terminal edge, so the loop's minimum lies in this triangle and
        // its byte is written here with the rest of the tile.
        const int L = (int)(f[j] & 3u), a = L == 2 ? 0 : L + 1, b = L == 0 ? 2 : L - 1;
        const bool cand = (f[j] & kSeedBit) && fbit(f[j], a) && fbit(f[j], b);
        const int g = L == 0 ? tw[j][0] : (L == 1 ? tw[j][1] : tw[j][2]);
        const int tp = tri_of(g < 0 ? 0 : g), Lp = g - 3 * tp;
        const int ap = Lp == 2 ? 0 : Lp + 1, bp = Lp == 0 ? 2 : Lp - 1;
        const int kp = tp - base;
        const bool inp = (unsigned)kp < (unsigned)cnt;
        const uint32_t fp = s_f[inp ? kp : 0];
        bool quad = fbit(fp, ap) && fbit(fp, bp);
        if (cand && g >= 0 && !inp)   // partner outside the tile (rare on ordered meshes)
            quad = outside_fbit(T, 3 * tp + ap, Lp) && outside_fbit(T, 3 * tp + bp, Lp);
        const uint8_t code = !cand ? (uint8_t)0
                             : g < 0 ? loop_code(h0, 3)
                             : !quad ? (uint8_t)0
                             : tp == t + 1 ? (uint8_t)((kPlQuadNext << 2) | Lp)
                                           : loop_code(h0 + min(a, b), 4);
        openmask |= ((f[j] & kSeedBit) && !code) ? 1 << j : 0;
        s_pl[lt] = code;   // entries past cnt are never stored
        codes[j] = code;
        scnt += code ? 1 : 0;
        slen += !code ? 0 : (code >> 2) == kPlQuadNext ? 4 : (code >> 2);
    }
    // One block scan places the turns still open in the LDS queue and the
    // open seeds in the walk list (stripe by tile, one atomic per block), and
    // totals the loops settled here for their compaction tile.  Each count
    // fits in 16 bits (at most 2 per triangle, lengths at most 4 per
    // triangle, tiles of at most 1024 triangles), so two ride in one int.
    {
        __shared__ int s_scan[72];
        __shared__ int s_wbase;
        int ea, eb, ta, tb;
        block_excl_scan2((__popc(pend) << 16) | __popc(openmask), (scnt << 16) | slen, ea, eb, ta, tb, s_scan);
        int eq = ea >> 16;
        const int eo = ea & 0xffff, tq = ta >> 16, to = ta & 0xffff;
        const int stripe = tile % kStripes;
        // the block's triangles lie in one compaction tile unless that tile is
        // smaller than this one or not aligned with it
        const bool one = base / cmp_tb == (base + cnt - 1) / cmp_tb;
        if (tid == 0) {
            s_wbase = to > 0 ? atomicAdd(&walk_counts[stripe * kStripePad], to) : 0;
            if (one && tb != 0)
                atomicAdd(reinterpret_cast<unsigned long long *>(agg + d.cmp_tile0 + base / cmp_tb),
                          ((unsigned long long)(uint32_t)(tb >> 16) << 32) | (unsigned long long)(tb & 0xffff));
        }
        const int ct0 = base / cmp_tb;   // first compaction tile of this tile
        if (!one) {   // totals per compaction tile in LDS, one global atomic each below
#pragma unroll
            for (int j = 0; j < ITEMS; j++) {
                if (!codes[j]) continue;
                const int k = (base + j * B + tid) / cmp_tb - ct0;
                const int len = (codes[j] >> 2) == kPlQuadNext ? 4 : (codes[j] >> 2);
                atomicAdd(&s_aggc[k], 1);
                atomicAdd(&s_aggl[k], len);
            }
        }
#pragma unroll
        for (int k = 0; k < 2 * ITEMS; k++) {
            qslot[k] = -1;
            if (!((pend >> k) & 1u)) continue;
            if (eq < qcap) {
                s_q[2 * eq] = cur[k];
                s_q[2 * eq + 1] = (src[k] << 3) | ((k & 1) == 0 ? 4 : 0) | (lab[k] + 1);
                qslot[k] = eq;
                pend &= ~(1u << k);
            }
            ++eq;
        }
        __syncthreads();
        if (!one && tid <= (base + cnt - 1) / cmp_tb - ct0 && s_aggc[tid] != 0)
            atomicAdd(reinterpret_cast<unsigned long long *>(agg + d.cmp_tile0 + ct0 + tid),
                      ((unsigned long long)(uint32_t)s_aggc[tid] << 32) | (unsigned long long)(uint32_t)s_aggl[tid]);
        const int wbase = s_wbase;
        err |= wbase + to > walk_cap;
        int e = stripe * walk_cap + wbase + eo;
        const int lim = (stripe + 1) * walk_cap;
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            if (!((openmask >> j) & 1)) continue;
            if (e < lim) {
                const int t = base + j * B + tid;
                walk[e].mesh = mi;
                walk[e].he = 3 * t + (int)(f[j] & 3u);
            }
            ++e;
        }
        // the queued turns, one per thread: only the first lanes of the block work
        const int nq = min(tq, qcap);
        for (int q = tid; q < nq; q += B) {
            const int w = s_q[2 * q + 1], sh = w >> 3;
            const bool nxt = (w & 4) != 0;
            const int res = run_turn(T, s_q[2 * q], (w & 3) - 1, nxt);
            err |= res < 0;
            s_q[2 * q] = res;   // the owner picks it up after the barrier
            if (nxt && res >= 0 && res == s_tw[sh])
                tile_tip(s_tip, &s_ntip, tcap, sh, base, rc, tips, cap_tips, d, mi, err);
        }
    }
    // turns beyond the queue (meshes whose polygons are mostly large), in registers
    for (int step = 0; pend; step++) {
#pragma unroll
        for (int k = 0; k < 2 * ITEMS; k++) {
            if (!((pend >> k) & 1u)) continue;
            const int r = step < kRotGuard ? turn_step(T, cur[k], lab[k], (k & 1) == 0) : -1;
            if (r == 0) continue;
            const int res = r > 0 ? cur[k] : -1;
            err |= r < 0;
            const int li = src[k] % 3;
            if ((k & 1) == 0) {
#pragma unroll
                for (int i = 0; i < 3; i++)
                    if (i == li) nv3[k >> 1][i] = res;
                if (res >= 0 && res == s_tw[src[k]])
                    tile_tip(s_tip, &s_ntip, tcap, src[k], base, rc, tips, cap_tips, d, mi, err);
            } else {
#pragma unroll
                for (int i = 0; i < 3; i++)
                    if (i == li) pv3[k >> 1][i] = res;
            }
            pend &= ~(1u << k);
        }
    }
    __syncthreads();
    // next'/prev' of this lane's triangles, with the queued turns' results
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const int lt = j * B + tid;
        if (lt >= cnt) continue;
#pragma unroll
        for (int kk = 0; kk < 2; kk++) {
            const int k = 2 * j + kk;
            if (qslot[k] < 0) continue;
            const int res = s_q[2 * qslot[k]], li = src[k] - 3 * lt;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                if (i != li) continue;
                if (kk == 0)
                    nv3[j][i] = res;
                else
                    pv3[j][i] = res;
            }
        }
        const int h0 = 3 * (base + lt);
        const v3i nv = v3i{nv3[j][0], nv3[j][1], nv3[j][2]}, pv = v3i{pv3[j][0], pv3[j][1], pv3[j][2]};
        if (NT) {
            __builtin_nontemporal_store(nv, reinterpret_cast<GLOBAL v3i *>(nxo + h0));
            __builtin_nontemporal_store(pv, reinterpret_cast<GLOBAL v3i *>(pvo + h0));
        } else {
            *reinterpret_cast<GLOBAL v3i *>(nxo + h0) = nv;
            *reinterpret_cast<GLOBAL v3i *>(pvo + h0) = pv;
        }
    }
    // the tile's label and loop bytes in whole words (the label bytes keep
    // their longest-edge bits, which other tiles may be reading)
    store_bytes_from_lds((gu8)(d.pl) + base, s_pl, cnt);
    store_bytes_from_lds(tflag + base, s_f, cnt);
    if (tid == 0) {   // the tile's tips: one append
        const int n = min(s_ntip, tcap);
        if (n > 0) {
            const int at = atomicAdd(&rc->ntips, n);
            atomicAdd(&d.ctr->ntips, n);
            for (int i = 0; i < n; i++) {
                if (at + i < cap_tips) {
                    tips[at + i].mesh = mi;
                    tips[at + i].he = 3 * base + s_tip[i];
                } else {
                    err = true;
                }
            }
        }
    }
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
            const TwinView twin = twin_view(d);
            // a: the only frontier edge at the tip v = target(e.he), leaving v.
            // The middle edge is the outgoing half-edge floor(deg / 2)
            // clockwise steps from a.  Turning clockwise (c) and counter-
            // clockwise (b) from a at once, the two meet there after about
            // deg / 2 steps: c one step short of b after k steps means deg =
            // 2k + 1 and the middle is c; c and b equal after k + 1 steps
            // means deg = 2k + 2 and the middle is that half-edge.
            a = twin[e.he];
            bool err = a < 0;
            if (!err) {
                int c = a, b = a;
                for (int k = 0;; k++) {
                    const int gc = twin[c], gb = twin[he_prev(b)];   // both loads in flight
                    if (gc < 0 || gb < 0 || k > kRotGuard) {
                        err = true;
                        break;
                    }
                    const int c1 = he_next(gc);
                    if (c1 == b && k > 0) {   // odd degree
                        m = c;
                        break;
                    }
                    if (c1 == gb) {   // even degree
                        m = c1;
                        break;
                    }
                    c = c1;
                    b = gb;
                }
                if (!err) {
                    mt = twin[m];
                    err = mt < 0;
                }
            }
            if (err) {
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

// One lane per anchor o0 (a half-edge leaving a vertex x at either end of a
// new frontier edge) takes next'/prev' around x again in one sweep.  Around
// x, the outgoing half-edge o is preceded in its triangle by prev(o), which
// enters x; next' of a frontier prev(o) is the nearest frontier outgoing
// half-edge at o or clockwise after it, and prev' is its inverse.  So a
// sweep counter-clockwise (o <- twin(prev(o))) from a frontier outgoing
// half-edge, keeping the last frontier outgoing half-edge it passed, sets
// them all with one dependent load per step.  A vertex on the boundary is
// swept from where the clockwise search stopped to the counter-clockwise
// end, then from the clockwise end back.  Anchors at one vertex write the
// same values.
__device__ __forceinline__ void sweep_step(gcu8 tfl, gint nxo, gint pvo, int o, int &cur) {
    const int t = tri_of(o), pin = he_prev(o);
    const uint32_t f = tfl[t];
    if (fbit(f, o - 3 * t)) cur = o;
    if (fbit(f, pin - 3 * t)) {
        nxo[pin] = cur;
        pvo[cur] = pin;
    }
}

__global__ void __launch_bounds__(256) k_fixup(const MeshDesc *__restrict__ descs, RunCounters *rc,
                                               const ListEntry *fixes, int cap_fix) {
    const int nfix = min(rc->nfix, cap_fix);
    const int stride = gridDim.x * blockDim.x;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nfix; q += stride) {
        const ListEntry en = fixes[q];
        const MeshDesc &d = descs[en.mesh];
        const TwinView twin = twin_view(d);
        const gcu8 tfl = (gcu8)d.tflag;
        const gint nxo = (gint)d.next_o, pvo = (gint)d.prev_o;
        bool ok = true;
        // clockwise from the anchor to a frontier outgoing half-edge (at the
        // latest the boundary one: boundary edges are frontier edges)
        int of = en.he;
        for (int k = 0;; k++) {
            if (is_frontier(d.tflag, of)) break;
            const int g = twin[of];   // a non-frontier edge is interior
            if (g < 0 || k > kRotGuard) {
                ok = false;
                break;
            }
            of = he_next(g);
            if (of == en.he) {   // no frontier edge at x: not an end of a middle edge
                ok = false;
                break;
            }
        }
        bool open = false;
        if (ok) {   // counter-clockwise from of, round to of or to the boundary
            int cur = of, o = of;
            for (int k = 0;; k++) {
                const int g = twin[he_prev(o)];
                sweep_step(tfl, nxo, pvo, o, cur);
                if (g < 0) {
                    open = true;
                    break;
                }
                o = g;
                if (o == of) break;
                if (k > kRotGuard) {
                    ok = false;
                    break;
                }
            }
        }
        if (ok && open && twin[of] >= 0) {   // the half-edges clockwise of of: from the clockwise end back to of
            int ob = of;
            for (int k = 0;; k++) {
                const int g = twin[ob];
                if (g < 0) break;
                ob = he_next(g);
                if (k > kRotGuard) {
                    ok = false;
                    break;
                }
            }
            int cur = ob, o = ob;
            for (int k = 0; ok && o != of; k++) {
                sweep_step(tfl, nxo, pvo, o, cur);
                const int g = twin[he_prev(o)];
                if (g < 0 || k > kRotGuard) {
                    ok = false;
                    break;
                }
                o = g;
            }
        }
        if (!ok) atomicOr(&d.ctr->err, kErrCorrupt);
    }
}

// ---------------------------------------------------------------------------
// k_walk: seed -> frontier half-edge -> loop minimum and length
// ---------------------------------------------------------------------------

// From seed s, turn clockwise around origin(s) until a frontier half-edge.
__device__ __forceinline__ int seek_frontier(const MeshDesc &d, int s) {
    int f = s;
    for (int k = 0; k < kRotGuard; k++) {
        if (is_frontier(d.tflag, f)) return f;
        const int g = twin_view(d)[f];
        if (g < 0) return -1;
        f = he_next(g);
    }
    return -1;
}


// Every entry of the walk list: from the seed to a frontier half-edge of its
// polygon (a frontier half-edge of the seed's own triangle if it has one),
// around the loop, and the loop recorded.  A loop still open after
// kWalkBoth steps (or after the first, when the loops are few and so
// latency decides) is walked from both ends from then on:
// forward along next' and backward along prev' from the start, the two
// loads of a step in flight together, until the ends meet, so a long loop
// of len half-edges takes about len / 2 dependent steps (short loops, the
// most, read no prev').  Each
// thread keeps ITEMS loops in flight and advances them in lock-step.  Every
// chain also writes the half-edges it visits to an LDS buffer (forward ones
// from the front, backward ones from the back), so the walker that claims a
// loop of at most BUF half-edges copies it to the scratch pool (rotation
// index of the minimum, then the half-edges in loop order from the first
// backward one) and k_compact places it without walking it again.  Whole
// waves iterate together: the pool is reserved once per wave and step, for
// every loop that closed in that step and fits the buffer, while the claims
// are still in flight (a walker that loses the claim leaves its space
// unused).
constexpr int kWalkBoth = 8;

template <int ITEMS, int BUF>
__global__ void __launch_bounds__(256) k_walk(const MeshDesc *__restrict__ descs, const ListEntry *walk,
                                              const int32_t *walk_counts, int walk_cap, uint64_t *agg,
                                              int cmp_tb, int32_t *wbuf, int32_t *wbuf_counts, int wbuf_cap) {
    constexpr int kSlots = 256 * ITEMS;
    __shared__ int s_pref[kStripes + 1];
    __shared__ int s_buf[BUF * kSlots];   // element k of chain slot q at k * kSlots + q
    const int total = striped_prefix(walk_counts, walk_cap, s_pref);
    const int nthreads = gridDim.x * blockDim.x;
    const int lane = __lane_id(), tid = threadIdx.x;
    const int wstripe = ((blockIdx.x * blockDim.x + tid) >> 6) % kStripes;   // this wave's pool stripe
    // few loops (a quarter of the threads or fewer): every walk is its own
    // critical path, so all go both ways from the first step; otherwise only
    // the long ones
    const int both = total <= nthreads / 4 ? 1 : kWalkBoth;
    for (int b0 = blockIdx.x * blockDim.x; b0 < total; b0 += nthreads * ITEMS) {   // block-uniform
        gcint nx[ITEMS], pv[ITEMS];
        // forward end fc (fa half-edges taken, from the start on), backward
        // end bc (bb taken before the start; the start itself while bb == 0);
        // the minimum so far and where: forward index, or ~backward index
        int mesh[ITEMS], fc[ITEMS], bc[ITEMS], fa[ITEMS], bb[ITEMS], mn[ITEMS], mpos[ITEMS], lim[ITEMS];
        bool live[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            fc[j] = bc[j] = mn[j] = -1;
            fa[j] = bb[j] = mpos[j] = lim[j] = 0;
            mesh[j] = 0;
            live[j] = false;
            nx[j] = pv[j] = nullptr;
            const int g = b0 + tid + j * nthreads;
            if (g >= total) continue;
            const ListEntry e = walk[striped_index(s_pref, walk_cap, g)];
            const MeshDesc &d = descs[e.mesh];
            mesh[j] = e.mesh;
            nx[j] = (gcint)d.next_o;
            pv[j] = (gcint)d.prev_o;
            lim[j] = 3 * d.nt;
            const int t = tri_of(e.he);
            const uint32_t f = ((gcu8)d.tflag)[t];
            int st = fbit(f, e.he - 3 * t) ? e.he : -1;
#pragma unroll
            for (int i = 0; i < 3; i++)
                if (st < 0 && fbit(f, i)) st = 3 * t + i;
            if (st < 0) st = seek_frontier(d, e.he);
            if (st < 0) {
                atomicOr(&d.ctr->err, kErrCorrupt);
                continue;
            }
            fc[j] = bc[j] = mn[j] = st;
            fa[j] = 1;
            live[j] = true;
            s_buf[j * 256 + tid] = st;
        }
        while (true) {
            bool active = false;
            int need[ITEMS], len[ITEMS], rot[ITEMS];
            bool closed[ITEMS];
            uint32_t claim[ITEMS];
#pragma unroll
            for (int j = 0; j < ITEMS; j++) {
                need[j] = len[j] = rot[j] = 0;
                closed[j] = false;
                claim[j] = 0;
                if (!live[j]) continue;
                const bool two = fa[j] >= both;
                const int nf = nx[j][fc[j]], nb = two ? pv[j][bc[j]] : 0;
                bool done = nf == bc[j];   // the forward end reached the backward one
                if (!done && nf >= 0) {
                    fc[j] = nf;
                    if (fa[j] < BUF) s_buf[fa[j] * kSlots + j * 256 + tid] = nf;
                    if (nf < mn[j]) {
                        mn[j] = nf;
                        mpos[j] = fa[j];
                    }
                    ++fa[j];
                    done = two && nb == nf;   // the backward end reached the forward one
                    if (two && !done && nb >= 0) {
                        bc[j] = nb;
                        if (bb[j] < BUF) s_buf[(BUF - 1 - bb[j]) * kSlots + j * 256 + tid] = nb;
                        if (nb < mn[j]) {
                            mn[j] = nb;
                            mpos[j] = ~bb[j];
                        }
                        ++bb[j];
                    }
                }
                len[j] = fa[j] + bb[j];
                if (nf < 0 || nb < 0 || len[j] > lim[j]) {
                    atomicOr(&descs[mesh[j]].ctr->err, kErrCorrupt);
                    live[j] = false;
                    continue;
                }
                if (done) {
                    closed[j] = true;
                    // position of the minimum in loop order from the first backward half-edge
                    rot[j] = mpos[j] >= 0 ? bb[j] + mpos[j] : bb[j] - 1 - ~mpos[j];
                    claim[j] = claim_issue(descs[mesh[j]], mn[j], len[j]);
                    // whole 16-byte groups, so k_compact reads a loop with vector loads
                    need[j] = len[j] <= BUF ? (len[j] + 4) & ~3 : 0;
                    live[j] = false;
                    continue;
                }
                active = true;
            }
            // pool space for the loops claimed in this step: one atomic per wave
            int mine = 0;
#pragma unroll
            for (int j = 0; j < ITEMS; j++) mine += need[j];
            const int incl = wave_incl_scan(mine);   // the loop's exit is wave-uniform: all lanes here
            const int wtot = __builtin_amdgcn_readlane(incl, kWave - 1);
            int wbase = 0;
            if (lane == 0 && wtot > 0) wbase = atomicAdd(&wbuf_counts[wstripe * kStripePad], wtot);
            wbase = __builtin_amdgcn_readlane(wbase, 0);
            const bool room = wbase + wtot <= wbuf_cap;
            int pos = wstripe * wbuf_cap + wbase + incl - mine;
#pragma unroll
            for (int j = 0; j < ITEMS; j++) {
                if (!closed[j]) continue;
                const MeshDesc &d = descs[mesh[j]];
                const bool won = claim_won(d, claim[j], mn[j], len[j], agg, cmp_tb);
                // a loop too long for its length code is never stored, so its
                // minimum's lpos slot is free: its length goes there for k_compact
                if (won && len[j] >= kPlMax) ((gint)d.lpos)[tri_of(mn[j])] = len[j];
                if (won && need[j] && room) {
                    const gint out = (gint)wbuf + pos;
                    out[0] = rot[j];
                    // the backward half-edges (from the back of the buffer), then the forward ones
                    for (int k = 0; k < len[j]; k++) {
                        const int at = k < bb[j] ? BUF - bb[j] + k : k - bb[j];
                        out[1 + k] = s_buf[at * kSlots + j * 256 + tid];
                    }
                    const int tm = tri_of(mn[j]);
                    ((gint)d.lpos)[tm] = pos;
                    atomicOr(reinterpret_cast<uint32_t *>(d.tflag) + (tm >> 2), kStoredBit << (8 * (tm & 3)));
                }
                pos += need[j];
            }
            if (!__any(active)) break;
        }
    }
}

// The loops k_compact left out, each written from its minimum at its offset
// from both ends at once: position s forward along next' and position len - s
// backward along prev', so the two loads of a step are in flight together and
// a loop of len half-edges takes about len / 2 dependent steps.
template <int ITEMS>
__global__ void __launch_bounds__(256) k_emit(const MeshDesc *__restrict__ descs, const EmitEntry *emit,
                                              const int32_t *emit_counts, int emit_cap) {
    __shared__ int s_pref[kStripes + 1];
    const int total = striped_prefix(emit_counts, emit_cap, s_pref);
    const int nthreads = gridDim.x * blockDim.x;
    for (int g0 = blockIdx.x * blockDim.x + threadIdx.x; g0 < total; g0 += nthreads * ITEMS) {
        gcint nx[ITEMS], pv[ITEMS];
        gint out[ITEMS];
        int mesh[ITEMS], f[ITEMS], b[ITEMS], len[ITEMS];
        bool live[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            live[j] = false;
            f[j] = b[j] = len[j] = mesh[j] = 0;
            nx[j] = pv[j] = nullptr;
            out[j] = nullptr;
            const int g = g0 + j * nthreads;
            if (g >= total) continue;
            const EmitEntry e = emit[striped_index(s_pref, emit_cap, g)];
            const MeshDesc &d = descs[e.mesh];
            mesh[j] = e.mesh;
            // k_compact left the loop's length in its first slot
            const int L = (e.off >= 0 && e.off < 3 * d.nt) ? ((gcint)d.loop_he)[e.off] : -1;
            if (L < 1 || (long long)e.off + L > 3ll * d.nt) {
                atomicOr(&d.ctr->err, kErrCorrupt);
                continue;
            }
            nx[j] = (gcint)d.next_o;
            pv[j] = (gcint)d.prev_o;
            out[j] = (gint)d.loop_he + e.off;
            f[j] = b[j] = e.mn;
            len[j] = L;
            out[j][0] = e.mn;
            live[j] = L > 1;
        }
        for (int s = 1;; s++) {
            bool active = false;
#pragma unroll
            for (int j = 0; j < ITEMS; j++) {
                if (!live[j]) continue;
                const int bi = len[j] - s;   // the backward end's position; the forward end's is s
                if (s > bi) {
                    live[j] = false;
                    continue;
                }
                const int nf = nx[j][f[j]], nb = pv[j][b[j]];   // both in flight together
                if (nf < 0 || nb < 0) {
                    atomicOr(&descs[mesh[j]].ctr->err, kErrCorrupt);
                    live[j] = false;
                    continue;
                }
                out[j][s] = nf;
                if (s < bi) out[j][bi] = nb;
                f[j] = nf;
                b[j] = nb;
                active = true;
            }
            if (!active) break;
        }
    }
}

// ---------------------------------------------------------------------------
// k_tile_scan: exclusive scan of the compaction tiles' loop totals
//
// k_relink (settled loops) and k_walk (walked loops) add every loop, once, to
// the total of the compaction tile holding its minimum: (loops << 32 |
// half-edges).  One block per mesh turns the totals into exclusive prefixes
// in place and records the mesh's polygon and loop half-edge counts, so each
// k_compact tile starts with its output offsets known.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(1024) k_tile_scan(const MeshDesc *__restrict__ descs, uint64_t *status,
                                                     uint64_t *cpre, int cmp_tb) {
    // block (mesh, chunk): tiles [chunk * kScanChunk, ...) of that mesh,
    // kTileScanItems consecutive ones per thread, read and written contiguously
    __shared__ int s_scan[72];
    __shared__ int s_last;
    const MeshDesc &d = descs[blockIdx.x];
    const int ntiles = d.nt > 0 ? (d.nt + cmp_tb - 1) / cmp_tb : 1;
    const int nchunks = (ntiles + kScanChunk - 1) / kScanChunk;
    const int chunk = blockIdx.y;
    if (chunk >= nchunks) return;   // the whole block
    const int tid = threadIdx.x, k0 = chunk * kScanChunk + tid * kTileScanItems;
    uint64_t *st = status + d.cmp_tile0;
    uint64_t v[kTileScanItems];
    int lc = 0, lh = 0;
#pragma unroll
    for (int i = 0; i < kTileScanItems; i++) {
        v[i] = k0 + i < ntiles ? st[k0 + i] : 0ull;
        lc += (int)(v[i] >> 32);
        lh += (int)(uint32_t)v[i];
    }
    int ec, eh, tc, th;
    block_excl_scan2(lc, lh, ec, eh, tc, th, s_scan);
#pragma unroll
    for (int i = 0; i < kTileScanItems; i++) {
        if (k0 + i < ntiles) st[k0 + i] = ((uint64_t)(uint32_t)ec << 32) | (uint32_t)eh;
        ec += (int)(v[i] >> 32);
        eh += (int)(uint32_t)v[i];
    }
    if (nchunks == 1) {   // (uniform) the whole mesh in one block: its totals at once
        if (tid == 0) {
            cpre[d.cmp_tile0] = 0ull;
            const bool ok = tc >= 0 && th >= 0 && tc <= d.nt && th <= 3 * d.nt;
            d.ctr->npoly = ok ? tc : 0;
            d.ctr->nloop = ok ? th : 0;
            if (ok)
                d.loop_off[tc] = th;
            else
                atomicOr(&d.ctr->err, kErrCorrupt);
        }
        return;
    }
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


template <int ITEMS>
__global__ void __launch_bounds__(1024) k_compact(const MeshDesc *__restrict__ descs, int nmesh,
                                                  const uint64_t *status, const uint64_t *cpre, EmitEntry *emit,
                                                  int32_t *emit_counts, int emit_cap, const int32_t *wbuf) {
    // LDS: loop half-edges (compact_he_cap of them), seeds and local offsets
    // (one per triangle)
    extern __shared__ int4 lds_raw[];
    const int B = blockDim.x, tid = threadIdx.x;
    const int TB = B * ITEMS;
    const int he_cap = compact_he_cap(TB);
    int *s_he = reinterpret_cast<int *>(lds_raw);
    int *s_seed = s_he + he_cap;
    int *s_off = s_seed + TB;
    __shared__ int s_scan[72];
    __shared__ int s_ebase;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int mi = find_mesh<2>(descs, nmesh, tile);
    const MeshDesc &d = descs[mi];
    const int nt = d.nt, nh = 3 * nt;
    const int ltile = tile - d.cmp_tile0;
    const int mesh_tiles = nt > 0 ? (nt + TB - 1) / TB : 1;
    const int t0 = ltile * TB + tid * ITEMS;
    const gcint nx = (gcint)d.next_o;
    const gcu8 plb = (gcu8)d.pl, tfl = (gcu8)d.tflag;
    // prefix within the chunk plus the chunk's prefix (no field carries)
    const uint64_t pre = status[tile] + cpre[d.cmp_tile0 + ltile / kScanChunk * kScanChunk];
    const int pc = (int)(pre >> 32), ps = (int)(uint32_t)pre;

    // 1. loop minima and lengths of this thread's ITEMS contiguous triangles;
    //    which loops are longer than a quad, and which of those k_walk stored
    //    (the rest k_emit writes)
    //    (the walk-pool positions come with them, read whether or not a loop
    //    was stored there, so a stored loop's pool read follows directly)
    uint8_t code[ITEMS], fl[ITEMS];
    int lp[ITEMS];
    const gcint lpos = (gcint)d.lpos;
    if (ITEMS == 4 && t0 + 4 <= nt) {
        const uint32_t w = *reinterpret_cast<GLOBAL const uint32_t *>(plb + t0);
        const uint32_t v = *reinterpret_cast<GLOBAL const uint32_t *>(tfl + t0);
        const v4i l4 = *(GLOBAL const v4i *)(lpos + t0);
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            code[j] = (uint8_t)(w >> (8 * (j & 3)));
            fl[j] = (uint8_t)(v >> (8 * (j & 3)));
        }
        lp[0] = l4.x;
        lp[1 % ITEMS] = l4.y;
        lp[2 % ITEMS] = l4.z;
        lp[3 % ITEMS] = l4.w;
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            code[j] = t0 + j < nt ? plb[t0 + j] : 0;
            fl[j] = t0 + j < nt ? tfl[t0 + j] : 0;
            lp[j] = t0 + j < nt ? lpos[t0 + j] : 0;
        }
    }
    int lens[ITEMS];
    bool defer[ITEMS];
    int cnt = 0, sum = 0, nd = 0;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        lens[j] = 0;
        defer[j] = false;
        if (!code[j]) continue;
        int len = code[j] >> 2;
        if (len == kPlQuadNext) len = 4;
        // longer than the code holds: k_walk left the length in lpos
        if (len >= kPlMax) len = lp[j] >= kPlMax && lp[j] <= nh ? lp[j] : -1;
        if (len <= 0) {
            bad = true;
            len = 0;
        }
        lens[j] = len;
        // loops of three and two-triangle loops of four are written here
        defer[j] = len > 0 && len != 3 && !(len == 4 && __popc((fl[j] >> 2) & 7u) == 2);
        cnt += 1;
        sum += len;
        nd += defer[j] && !(fl[j] & kStoredBit);
    }
    // 2. block scan: tile-local loop index and offset, emit-list slot
    int ecn, esum, tcn, tsum;
    block_excl_scan2(cnt | (nd << 16), sum, ecn, esum, tcn, tsum, s_scan);
    const int tcnt = tcn & 0xffff, tnd = tcn >> 16;
    const int stripe = tile % kStripes;
    if (tid == 0) {
        s_ebase = tnd > 0 ? atomicAdd(&emit_counts[stripe * kStripePad], tnd) : 0;
        // the tiles' prefixes must add up to the mesh totals
        if (ltile == mesh_tiles - 1 && (pc + tcnt != d.ctr->npoly || ps + tsum != d.ctr->nloop)) bad = true;
    }
    const bool fits = tsum <= he_cap && pc + tcnt <= nt && ps + tsum <= nh;
    // 3. seeds, local offsets and loops; into LDS, or straight to global
    //    memory for a tile whose loops do not fit
    // A loop of 3 is one triangle: (mn, next, prev).  A loop of 4 is two
    // triangles: the minimum's triangle has frontier half-edges a, b = next(a)
    // and crosses to the other triangle at b, whose two frontier half-edges
    // follow as p1 = next'(b), next(p1).  Longer loops get their offset here
    // and are written by k_emit.
    __syncthreads();
    const int elim = (stripe + 1) * emit_cap;
    bad |= s_ebase + tnd > emit_cap;
    // the body is instantiated twice: loops into LDS (the tile fits, the
    // usual case), or straight to global memory; the tile decides for all
    // its threads
    auto place_loops = [&](auto he_out) {
    int q = ecn & 0xffff, off = esum, e = (ecn >> 16) + stripe * emit_cap + s_ebase;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        if (!code[j]) continue;
        const int t = t0 + j;
        const uint32_t fb = (fl[j] >> 2) & 7u;
        const bool qn = (code[j] >> 2) == kPlQuadNext;
        const int mn = 3 * t + (qn ? __builtin_ctz(fb | 8u) : (code[j] & 3));
        const bool place = fits || (pc + q < nt && ps + off + lens[j] <= nh);
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
            if (lens[j] == 3) {
                he_out[off] = mn;
                he_out[off + 1] = he_next(mn);
                he_out[off + 2] = he_prev(mn);
            } else if (!defer[j] && lens[j] == 4) {
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
            } else if (defer[j] && (fl[j] & kStoredBit)) {
                // stored by k_walk in walk order from some start; rotate so
                // the loop begins at its minimum (loads first, all in flight)
                static_assert(kWalkBuf % 4 == 0, "stored loops are read in 16-byte groups");
                const int len = lens[j];
                const GLOBAL v4i *src = (GLOBAL const v4i *)((gcint)wbuf + lp[j]);
                v4i g[kWalkBuf / 4 + 1];   // rotation index, then the half-edges
#pragma unroll
                for (int c = 0; c <= kWalkBuf / 4; c++) g[c] = src[c];
                int v[kWalkBuf + 4];
#pragma unroll
                for (int c = 0; c <= kWalkBuf / 4; c++) {
                    v[4 * c] = g[c].x;
                    v[4 * c + 1] = g[c].y;
                    v[4 * c + 2] = g[c].z;
                    v[4 * c + 3] = g[c].w;
                }
                const int rot = v[0];
                if (rot < 0 || rot >= len || len > kWalkBuf || v[1 + rot] != mn) bad = true;
                else
#pragma unroll
                    for (int k = 0; k < kWalkBuf; k++)
                        if (k < len) he_out[off + (k >= rot ? k - rot : k - rot + len)] = v[1 + k];
            } else if (defer[j]) {
                if (e < elim) {
                    emit[e].mesh = mi;
                    emit[e].mn = mn;
                    emit[e].off = ps + off;
                }
                // the loop's length in its own first slot, which k_emit reads
                // and then overwrites with the minimum
                he_out[off] = lens[j];
                ++e;
            }
        }
        ++q;
        off += lens[j];
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
        constexpr int kSeedIt = ITEMS;                  // tcnt <= TB
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
// k_small: the whole chain for one small mesh in one workgroup
//
// Below a few thousand triangles the chain's time is its eight launches and
// the memory round trips that open each of them, not its bytes.  A mesh of at
// most kSmallMaxTri triangles keeps every intermediate array in LDS, and one
// workgroup runs the steps with block barriers between them:
//   1. longest edge of every triangle (Section 6.1, Algorithm 8);
//   2. frontier half-edges (Section 6.2, Algorithm 9);
//   3. next' of every frontier half-edge by turning clockwise around its
//      target (Section 6.5, Algorithm 12).  The same turns find the barrier
//      tips (Section 6.4, Algorithm 11): a turn from next(h) that comes all
//      the way round to twin(h) met no other frontier edge, so the target of
//      h is a tip whose degree is the turn's length; its middle edge lies
//      half the degree further round from twin(h).  The turns around both
//      ends of every middle edge are then taken again with the repaired
//      frontier;
//   4. prev' as the inverse of next';
//   5. every half-edge's loop minimum and its distance to it along next', by
//      pointer doubling (Section 6.6, Algorithm 14): after a round with
//      window w, a half-edge holds the minimum of the w half-edges from it on
//      and how far ahead that minimum first occurs; a round that lowers no
//      minimum has reached each loop's minimum everywhere (the windows that
//      start w apart cover a loop and all hold the same minimum);
//   6. seeds, loop offsets and loops in half-edge order from a block scan
//      over the loop minima (Section 6.7).
// In LDS a half-edge 3t + i is slot 4t + i, so next and the triangle of a
// slot are bit operations (the order of slots is the order of half-edges),
// and a slot's 16-bit entry holds its twin's slot with both frontier bits.
// Each thread owns a few triangles and half-edges, and the turns of its
// items step together so that their LDS reads overlap.  The outputs equal
// the tiled chain's element by element.  One workgroup per mesh: a batch
// whose meshes are all small is one launch.
// ---------------------------------------------------------------------------

constexpr uint32_t kSlotNone = 0x3fff;   // no twin (4t + 3 is never a half-edge's slot)
constexpr uint32_t kSlotF1 = 1u << 14;   // frontier (label phase)
constexpr uint32_t kSlotF2 = 1u << 15;   // frontier after the repair
constexpr uint32_t kNone16 = 0xffff;     // no minimum (not on a loop)

__device__ __forceinline__ int slot_next(int q) { return (q & 3) == 2 ? q - 2 : q + 1; }
__device__ __forceinline__ int slot_prev(int q) { return (q & 3) == 0 ? q + 2 : q - 1; }
__device__ __forceinline__ int slot_he(int q) { return 3 * (q >> 2) + (q & 3); }

// IT: half-edges per thread (3, 6 or 12; meshes of up to IT * kSmallBlock / 3
// triangles), IT / 3 triangles per thread
// The counts of a run go to the mesh's device counters and, for a run
// launched on its own, straight to the caller's coherent host copy.
__device__ __forceinline__ void small_counts(const MeshDesc &d, MeshCounters *host, const MeshCounters &c) {
    if (d.ctr) *d.ctr = c;
    if (host) *host = c;
}

template <int IT>
__device__ __forceinline__ void small_body(const MeshDesc &d, MeshCounters *host) {
    constexpr int TI = IT / 3;
    extern __shared__ int4 lds_raw[];
    __shared__ int s_scan[72];
    __shared__ int s_cnt[4];   // tied maxima, tips, new middle edges, frontier half-edges
    const int nt = d.nt, nh = 3 * nt, tid = threadIdx.x;
    if (nt <= 0 || nt > TI * kSmallBlock) {   // (uniform) an empty mesh; larger ones are never launched here
        if (tid == 0) {
            MeshCounters c{};
            c.err = nt != 0 ? kErrCorrupt : 0;
            small_counts(d, host, c);
            if (nt == 0) d.loop_off[0] = 0;
        }
        return;
    }
    if (tid < 4) s_cnt[tid] = 0;
    char *base = reinterpret_cast<char *>(lds_raw);
    const size_t a16 = small_a16_bytes(nt);
    uint16_t *s_e = reinterpret_cast<uint16_t *>(base);             // twin slot | frontier bits
    uint16_t *s_p = s_e;                                             // then doubling pointer, loop offset
    uint16_t *s_nx = reinterpret_cast<uint16_t *>(base + a16);      // next', then loop length at minima
    uint32_t *s_mk = reinterpret_cast<uint32_t *>(base + 2 * a16);  // minimum | distance to it << 16
    uint8_t *s_lab = reinterpret_cast<uint8_t *>(base + 4 * a16);   // local index of the longest edge
    int bad = 0;

    // 1. longest edges; edge i of t runs from corner i to corner i + 1, and a
    //    tie at the maximum goes to the lower edge id min(h, twin h).  All the
    //    corner and twin loads first, then the coordinates.
    {
        const gcv2i xy = (gcv2i)(d.xy);
        const TwinView twin = twin_view(d);
        int v[TI][3], g[TI][3];
#pragma unroll
        for (int j = 0; j < TI; j++) {
            const int t = tid + j * kSmallBlock, tt = t < nt ? t : 0;
            if (!d.org8) {
                const gcint org = (gcint)(d.org);
#pragma unroll
                for (int i = 0; i < 3; i++) v[j][i] = org[3 * tt + i];
            } else {
                const v2i r = ((GLOBAL const v2i *)d.org8)[tt];
                const int d1 = (int)(int16_t)(r.y & 0xffff), d2 = r.y >> 16;
                v[j][0] = r.x;
                v[j][1] = d1 != kEsc16 ? r.x + d1 : esc_lookup(d.esc, d.esc_mask, ~(3 * tt + 1));
                v[j][2] = d2 != kEsc16 ? r.x + d2 : esc_lookup(d.esc, d.esc_mask, ~(3 * tt + 2));
            }
#pragma unroll
            for (int i = 0; i < 3; i++) g[j][i] = twin[3 * tt + i];
        }
        int2 p[TI][3];
#pragma unroll
        for (int j = 0; j < TI; j++) {
            const bool in = tid + j * kSmallBlock < nt;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                const bool ok = v[j][i] >= 0 && v[j][i] < d.nv;
                bad |= in && !ok;
                const v2i q = xy[ok ? v[j][i] : 0];
                p[j][i] = make_int2(q.x, q.y);
            }
        }
        int ties = 0;
#pragma unroll
        for (int j = 0; j < TI; j++) {
            const int t = tid + j * kSmallBlock;
            if (t >= nt) continue;
            const long long l[3] = {sq_len(p[j][0], p[j][1]), sq_len(p[j][1], p[j][2]), sq_len(p[j][2], p[j][0])};
            int best = 0;
            long long bl = l[0];
            int bid = (g[j][0] >= 0 && g[j][0] < 3 * t) ? g[j][0] : 3 * t;
#pragma unroll
            for (int i = 1; i < 3; i++) {
                const int h = 3 * t + i, id = (g[j][i] >= 0 && g[j][i] < h) ? g[j][i] : h;
                if (l[i] > bl || (l[i] == bl && id < bid)) {
                    best = i;
                    bl = l[i];
                    bid = id;
                }
            }
            ties += (l[0] == bl) + (l[1] == bl) + (l[2] == bl) > 1;
            s_lab[t] = (uint8_t)best;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                const int gi = g[j][i];
                const bool ok = gi >= 0 && gi < nh;
                bad |= gi >= nh || gi < -1;
                s_e[4 * t + i] = (uint16_t)(ok ? 4 * tri_of(gi) + (gi - 3 * tri_of(gi)) : kSlotNone);
            }
        }
        if (ties) atomicAdd(&s_cnt[0], ties);
    }
    __syncthreads();

    // the half-edges this thread owns: h = tid + j * kSmallBlock, slot q[j]
    int q[IT];
#pragma unroll
    for (int j = 0; j < IT; j++) {
        const int h = tid + j * kSmallBlock;
        q[j] = h < nh ? 4 * tri_of(h) + (h - 3 * tri_of(h)) : -1;
    }

    // 2. frontier half-edges: on the boundary, or the longest edge of neither
    //    triangle (both bits; the repair adds to the second)
    uint32_t front = 0;   // bit j: q[j] is a frontier half-edge (label phase, then repaired)
    {
        uint32_t e[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) e[j] = q[j] >= 0 ? s_e[q[j]] : kSlotNone;
#pragma unroll
        for (int j = 0; j < IT; j++) {
            if (q[j] < 0) continue;
            const int g = (int)(e[j] & kSlotNone);
            const bool lh = s_lab[q[j] >> 2] == (q[j] & 3);
            const bool lg = g != (int)kSlotNone && s_lab[g >> 2] == (g & 3);
            const bool f = g == (int)kSlotNone || (!lh && !lg);
            if (f) {
                s_e[q[j]] = (uint16_t)(e[j] | kSlotF1 | kSlotF2);
                front |= 1u << j;
            }
        }
    }
    __syncthreads();

    // 3. turns: next'(h) = the first frontier slot clockwise around the target
    //    of h from next(h); a turn that ends at twin(h) found a tip
    int nx[IT], deg[IT];
    uint32_t tip = 0;
    {
        uint32_t act = front;
#pragma unroll
        for (int j = 0; j < IT; j++) {
            nx[j] = (front >> j) & 1u ? slot_next(q[j]) : 0;
            deg[j] = 1;
        }
        for (int it = 0; act && it <= 4 * nt; it++) {
            uint32_t e[IT];
#pragma unroll
            for (int j = 0; j < IT; j++) e[j] = ((act >> j) & 1u) ? s_e[nx[j]] : kSlotF1;
#pragma unroll
            for (int j = 0; j < IT; j++) {
                if (!((act >> j) & 1u)) continue;
                if (e[j] & kSlotF1) {
                    act &= ~(1u << j);
                } else if ((e[j] & kSlotNone) == kSlotNone) {   // a non-frontier edge on the boundary: not a valid mesh
                    act &= ~(1u << j);
                    bad = 1;
                } else {
                    nx[j] = slot_next((int)(e[j] & kSlotNone));
                    deg[j]++;
                }
            }
        }
        bad |= act != 0;
        int tips = 0, fresh = 0;
#pragma unroll
        for (int j = 0; j < IT; j++) {
            if (!((front >> j) & 1u)) continue;
            s_nx[q[j]] = (uint16_t)nx[j];
            const int tw = (int)(s_e[q[j]] & kSlotNone);
            if (tw == (int)kSlotNone || nx[j] != tw) continue;
            // a tip: its frontier half-edge is tw; the middle edge deg / 2
            // clockwise steps further
            int m = tw;
            for (int k = 0; k < deg[j] / 2; k++) m = slot_next((int)(s_e[m] & kSlotNone));
            const int mt = (int)(s_e[m] & kSlotNone);
            if (mt == (int)kSlotNone) {
                bad = 1;
                continue;
            }
            tip |= 1u << j;
            deg[j] = m;   // from here on: the tip's middle slot
            const int lo = min(m, mt), hi = max(m, mt);
            uint32_t *w32 = reinterpret_cast<uint32_t *>(s_e);
            const uint32_t blo = kSlotF2 << (16 * (lo & 1));
            const uint32_t old = atomicOr(&w32[lo >> 1], blo);
            atomicOr(&w32[hi >> 1], kSlotF2 << (16 * (hi & 1)));
            tips++;
            fresh += !(old & blo);   // the edge's first tip counts it
        }
        if (tips) {
            atomicAdd(&s_cnt[1], tips);
            atomicAdd(&s_cnt[2], fresh);
        }
    }
    __syncthreads();

    // 3b. the turns around both ends of every middle edge again, over the
    //     repaired frontier: every slot entering such a vertex.  (Two tips may
    //     share a vertex; they write the same values.)
    if (s_cnt[1] > 0) {   // (uniform)
        auto turn2 = [&](int c) {
            for (int k = 0; k <= 4 * nt; k++) {
                const uint32_t e = s_e[c];
                if (e & kSlotF2) return c;
                if ((e & kSlotNone) == kSlotNone) return -1;
                c = slot_next((int)(e & kSlotNone));
            }
            return -1;
        };
        auto fix_vertex = [&](int o0) {   // o0 leaves the vertex
            bool open = false;
            int o = o0;
            for (int k = 0; k <= 4 * nt; k++) {   // clockwise
                const int pin = slot_prev(o);
                if (s_e[pin] & kSlotF2) {
                    const int c = turn2(slot_next(pin));
                    bad |= c < 0;
                    s_nx[pin] = (uint16_t)(c < 0 ? 0 : c);
                }
                const int g = (int)(s_e[o] & kSlotNone);
                if (g == (int)kSlotNone) {
                    open = true;
                    break;
                }
                o = slot_next(g);
                if (o == o0) break;
            }
            if (!open) return;
            o = o0;
            for (int k = 0; k <= 4 * nt; k++) {   // counter-clockwise, to the other boundary edge
                const int g = (int)(s_e[slot_prev(o)] & kSlotNone);
                if (g == (int)kSlotNone) break;
                o = g;
                const int pin = slot_prev(o);
                if (s_e[pin] & kSlotF2) {
                    const int c = turn2(slot_next(pin));
                    bad |= c < 0;
                    s_nx[pin] = (uint16_t)(c < 0 ? 0 : c);
                }
            }
        };
#pragma unroll
        for (int j = 0; j < IT; j++) {
            if (!((tip >> j) & 1u)) continue;
            const int m = deg[j], mt = (int)(s_e[m] & kSlotNone);
            fix_vertex(m);    // m leaves the tip
            fix_vertex(mt);   // mt leaves the middle edge's other end
        }
        __syncthreads();
    }

    // 4. next' and prev' out (prev' is next' inverted); the doubling's first
    //    window: m = min(q, n1), distance 1 when n1 is the smaller, p =
    //    next'(n1).  A thread keeps its own items' values in registers.
    int m[IT], k[IT], p[IT];
    {
        const gint nxo = (gint)d.next_o, pvo = (gint)d.prev_o;
#pragma unroll
        for (int j = 0; j < IT; j++) {
            if (q[j] < 0) continue;
            if (s_e[q[j]] & kSlotF2) front |= 1u << j;   // the repair's middle edges
        }
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const int h = tid + j * kSmallBlock;
            m[j] = kNone16;
            k[j] = 0;
            p[j] = q[j] >= 0 ? q[j] : 0;
            if (q[j] < 0) continue;
            if ((front >> j) & 1u) {
                const int n1 = s_nx[q[j]], hn = slot_he(n1);
                nxo[h] = hn;
                pvo[hn] = h;
                m[j] = min(q[j], n1);
                k[j] = n1 < q[j] ? 1 : 0;
                p[j] = s_nx[n1];
            } else {
                nxo[h] = -1;
                pvo[h] = -1;
            }
        }
    }
    if (__syncthreads_or(bad)) {   // (uniform) no loop structure to follow; every read of s_e is done
        if (tid == 0) {
            MeshCounters c{};
            c.err = kErrCorrupt;
            small_counts(d, host, c);
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < IT; j++) {
        if (q[j] < 0) continue;
        s_mk[q[j]] = (uint32_t)m[j] | ((uint32_t)k[j] << 16);
        s_p[q[j]] = (uint16_t)p[j];
    }
    __syncthreads();

    // 5. doubling: each round reads its operands before any thread writes
    bool done = false;
    for (int round = 0, w = 2; round < 16 && !done; round++, w *= 2) {
        uint32_t mkq[IT];
        int pq[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) {
            mkq[j] = s_mk[p[j]];
            pq[j] = s_p[p[j]];
        }
        __syncthreads();
        int lowered = 0;
#pragma unroll
        for (int j = 0; j < IT; j++) {
            if (!((front >> j) & 1u)) continue;
            const int mq = (int)(mkq[j] & 0xffffu);
            if (mq < m[j]) {   // the minimum lies beyond this window: w + its distance from p
                m[j] = mq;
                k[j] = w + (int)(mkq[j] >> 16);
                s_mk[q[j]] = (uint32_t)m[j] | ((uint32_t)k[j] << 16);
                lowered = 1;
            }
            p[j] = pq[j];
            s_p[q[j]] = (uint16_t)pq[j];
        }
        done = !__syncthreads_or(lowered);
    }
    bad |= !done;

    // 6. loops in the order of their minima: each thread scans a contiguous
    //    run of slots; a minimum's loop is one longer than the distance from
    //    its successor back to it
    constexpr int QT = 4 * TI;   // slots per thread
    const int q0 = tid * QT;
    int len[QT];
    int cnt = 0, sum = 0;
#pragma unroll
    for (int r = 0; r < QT; r++) {
        const int s = q0 + r;
        len[r] = 0;
        if ((r & 3) != 3 && (s >> 2) < nt && (int)(s_mk[s] & 0xffffu) == s) {
            len[r] = (int)(s_mk[s_nx[s]] >> 16) + 1;
            cnt++;
            sum += len[r];
        }
    }
    int ec, es, tc, ts;
    block_excl_scan2(cnt, sum, ec, es, tc, ts, s_scan);
    // a loop has at least three half-edges, and each half-edge one loop
    const bool fits = tc <= nt && ts <= nh;
    bad |= !fits;
    if (fits) {
        const gint seeds = (gint)d.seeds, loff = (gint)d.loop_off;
#pragma unroll
        for (int r = 0; r < QT; r++) {
            if (!len[r]) continue;
            const int s = q0 + r;
            seeds[ec] = slot_he(s);
            loff[ec] = es;
            s_p[s] = (uint16_t)es;       // the loop's first slot
            s_nx[s] = (uint16_t)len[r];  // and its length, for step 7
            ec++;
            es += len[r];
        }
        if (tid == 0) loff[tc] = ts;
    }
    __syncthreads();

    // 7. every frontier half-edge into its loop's slot: the minimum first,
    //    then the others in next' order
    if (fits) {
        const gint lhe = (gint)d.loop_he;
        int off[IT], ln[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const int mc = ((front >> j) & 1u) ? m[j] : 0;
            off[j] = s_p[mc];
            ln[j] = s_nx[mc];
        }
        int nfront = 0;
#pragma unroll
        for (int j = 0; j < IT; j++) {
            if (!((front >> j) & 1u)) continue;
            nfront++;
            const int pos = k[j] == 0 ? 0 : ln[j] - k[j];
            if (pos < 0 || pos >= ln[j] || off[j] + pos >= ts) {
                bad = 1;
                continue;
            }
            lhe[off[j] + pos] = tid + j * kSmallBlock;
        }
        if (nfront) atomicAdd(&s_cnt[3], nfront);
    }
    const int anybad = __syncthreads_or(bad);
    if (tid == 0) {
        MeshCounters c{};
        // every frontier half-edge lies on exactly one loop
        c.err = (anybad || s_cnt[3] != ts) ? kErrCorrupt : 0;
        c.nties = s_cnt[0];
        c.ntips = s_cnt[1];
        c.nmiddle = s_cnt[2];
        c.npoly = tc;
        c.nloop = ts;
        small_counts(d, host, c);
    }
}

// a batch of small meshes: one workgroup per descriptor
template <int IT>
__global__ void __launch_bounds__(kSmallBlock) k_small(const MeshDesc *__restrict__ descs) {
    small_body<IT>(descs[blockIdx.x], nullptr);
}

// one small mesh, its descriptor passed by value and its counts written to
// host memory: a call that needs nothing staged before it or copied after it
template <int IT>
__global__ void __launch_bounds__(kSmallBlock) k_small_one(const MeshDesc d, MeshCounters *host) {
    small_body<IT>(d, host);
}

// ---------------------------------------------------------------------------
// k_small_jobs: build and mesh one small job per workgroup
//
// The half-edge build of Section 4.1-4.2 for a job small enough for LDS, in
// the order and with the error reports of the staged build kernels: every
// coordinate in [0, 2^30]; every corner index in [0, nv) and no zero-area
// triangle (exact int64 orientation test), clockwise triangles reordered
// counter-clockwise; then twins by bucketing the half-edges by origin and
// searching the target's bucket for the reverse edge, where two reverse
// edges, or a repeated directed edge without one, is non-manifold.  Errors
// keep the lowest (rank << 8 | code): coordinates first, then the lowest bad
// triangle, then the lowest non-manifold half-edge; the twins are matched
// only when the first checks pass.  The built structure goes to device
// scratch and the workgroup then meshes it as k_small does.
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long job_key(unsigned long long rank, int code) {
    return (rank << 8) | (unsigned long long)(-code);
}

size_t small_job_lds_bytes(int max_nv, int max_nt) {
    // corners (3 nt), bucket starts (nv + 1), fill cursors (nv), bucket (3 nt)
    const size_t build = 4 * (3 * (size_t)max_nt + (size_t)max_nv + 1 + (size_t)max_nv + 3 * (size_t)max_nt) + 64;
    const size_t mesh = small_lds_bytes(max_nt);
    return build > mesh ? build : mesh;
}

template <int IT>
__global__ void __launch_bounds__(kSmallBlock) k_small_jobs(const SmallJob *__restrict__ jobs) {
    extern __shared__ int4 lds_raw[];
    __shared__ unsigned long long s_key;
    __shared__ int s_flip;
    __shared__ int s_scan[72];
    const SmallJob &jd = jobs[blockIdx.x];
    const int nv = jd.nv, nt = jd.nt, nh = 3 * nt, tid = threadIdx.x;
    if (tid == 0) {
        s_key = ~0ull;
        s_flip = 0;
    }
    if (nv < 0 || nt < 0 || nv > kJobSmallV || nt > (IT / 3) * kSmallBlock) {   // (uniform) never launched so
        if (tid == 0) {
            jd.counts[8] = (int)(uint32_t)job_key(0, -1);
            jd.counts[9] = 0;
        }
        return;
    }
    int *s_org = reinterpret_cast<int *>(lds_raw);   // 3 nt corners, counter-clockwise
    int *s_vst = s_org + nh;                          // nv + 1 bucket starts
    int *s_cur = s_vst + nv + 1;                      // nv fill cursors
    int *s_bkt = s_cur + nv;                          // nh half-edges grouped by origin
    __syncthreads();
    // coordinates (and the mesh's own copy of them)
    for (int v = tid; v < nv; v += kSmallBlock) {
        const int2 p = jd.xy[v];
        if (jd.xy_out) jd.xy_out[v] = p;
        if (p.x < 0 || p.x > (1 << 30) || p.y < 0 || p.y > (1 << 30)) atomicMin(&s_key, job_key(0, -2));
    }
    // corners: indices, orientation, counter-clockwise order
    int flips = 0;
    for (int t = tid; t < nt; t += kSmallBlock) {
        int a = jd.tri[3 * t], b = jd.tri[3 * t + 1], c = jd.tri[3 * t + 2];
        if ((unsigned)a >= (unsigned)nv || (unsigned)b >= (unsigned)nv || (unsigned)c >= (unsigned)nv) {
            atomicMin(&s_key, job_key(1ull + t, -1));
            a = b = c = 0;
        } else {
            const int2 pa = jd.xy[a], pb = jd.xy[b], pc = jd.xy[c];
            const long long o = ((long long)pb.x - pa.x) * ((long long)pc.y - pa.y) -
                                ((long long)pb.y - pa.y) * ((long long)pc.x - pa.x);
            if (o == 0) {
                atomicMin(&s_key, job_key(1ull + t, -3));
            } else if (o < 0) {
                const int sw = b;
                b = c;
                c = sw;
                flips++;
            }
        }
        s_org[3 * t] = a;
        s_org[3 * t + 1] = b;
        s_org[3 * t + 2] = c;
    }
    if (flips) atomicAdd(&s_flip, flips);
    for (int v = tid; v <= nv; v += kSmallBlock) s_vst[v] = 0;
    __syncthreads();
    if (s_key != ~0ull) {   // (uniform) the inputs failed their checks: no twins
        if (tid == 0) {
            jd.counts[8] = (int)(uint32_t)s_key;
            jd.counts[9] = (int)(uint32_t)(s_key >> 32);
        }
        return;
    }
    // out-degrees, their exclusive scan (four vertices per thread), buckets
    for (int h = tid; h < nh; h += kSmallBlock) atomicAdd(&s_vst[s_org[h]], 1);
    __syncthreads();
    {
        constexpr int VP = (kJobSmallV + kSmallBlock - 1) / kSmallBlock;
        const int v0 = tid * VP;
        int dv[VP], sum = 0;
#pragma unroll
        for (int k = 0; k < VP; k++) {
            dv[k] = v0 + k < nv ? s_vst[v0 + k] : 0;
            sum += dv[k];
        }
        int ex, ex2, tot, tot2;
        block_excl_scan2(sum, 0, ex, ex2, tot, tot2, s_scan);
#pragma unroll
        for (int k = 0; k < VP; k++) {
            if (v0 + k < nv) {
                s_vst[v0 + k] = ex;
                s_cur[v0 + k] = ex;
            }
            ex += dv[k];
        }
        if (tid == 0) s_vst[nv] = tot;
    }
    __syncthreads();
    for (int h = tid; h < nh; h += kSmallBlock) s_bkt[atomicAdd(&s_cur[s_org[h]], 1)] = h;
    __syncthreads();
    // twins: h = u->v pairs with the one v->u in v's bucket
    for (int h = tid; h < nh; h += kSmallBlock) {
        const int u = s_org[h], v = s_org[he_next(h)];
        int found = -1, nrev = 0, ndup = 0;
        for (int k = s_vst[v], e = s_vst[v + 1]; k < e; k++) {
            const int g = s_bkt[k];
            if (s_org[he_next(g)] == u) {
                found = g;
                ++nrev;
            }
        }
        if (nrev == 0)
            for (int k = s_vst[u], e = s_vst[u + 1]; k < e; k++) {
                const int g = s_bkt[k];
                if (g != h && s_org[he_next(g)] == v) ++ndup;
            }
        if (nrev > 1 || ndup > 0) atomicMin(&s_key, job_key(1ull + nt + h, -4));
        jd.org[h] = u;
        jd.twin[h] = nrev == 1 ? found : -1;
    }
    __syncthreads();
    if (tid == 0) {
        jd.counts[8] = (int)(uint32_t)s_key;
        jd.counts[9] = (int)(uint32_t)(s_key >> 32);
        jd.counts[10] = s_flip;
    }
    if (s_key != ~0ull || jd.build_only) return;   // (uniform)
    __threadfence_block();   // the structure in global memory, for the meshing that follows
    MeshDesc d{};
    d.xy = jd.xy;
    d.org = jd.org;
    d.twin = jd.twin;
    d.next_o = jd.next_o;
    d.prev_o = jd.prev_o;
    d.seeds = jd.seeds;
    d.loop_off = jd.loop_off;
    d.loop_he = jd.loop_he;
    d.ctr = reinterpret_cast<MeshCounters *>(jd.counts);
    d.nt = nt;
    d.nv = nv;
    small_body<IT>(d, nullptr);
}

hipError_t launch_small_jobs(const SmallJob *jobs, int n, int max_nv, int max_nt, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 grid(n), block(kSmallBlock);
    const size_t lds = small_job_lds_bytes(max_nv, max_nt);
    if (max_nt <= kSmallBlock)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_small_jobs<3>), grid, block, lds, s, jobs);
    else if (max_nt <= 2 * kSmallBlock)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_small_jobs<6>), grid, block, lds, s, jobs);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_small_jobs<12>), grid, block, lds, s, jobs);
    return hipGetLastError();
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

template <bool CM, bool NT>
hipError_t launch_relink_nt(const LaunchCfg &cfg, const RunBuffers &rb, hipStream_t s, size_t lds, int cmp_tb) {
    const dim3 grid(rb.he_tiles), block(cfg.block_relink);
#define GP_RELINK_ARGS rb.descs, rb.nmesh, rb.rc, rb.tips, rb.cap_tips, rb.walk, rb.walk_counts, rb.walk_cap, \
                       rb.status, cmp_tb
    switch (cfg.items_relink) {
        case 1: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_relink<1, CM, NT>), grid, block, lds, s, GP_RELINK_ARGS); break;
        case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_relink<2, CM, NT>), grid, block, lds, s, GP_RELINK_ARGS); break;
        case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_relink<4, CM, NT>), grid, block, lds, s, GP_RELINK_ARGS); break;
        case 8: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_relink<8, CM, NT>), grid, block, lds, s, GP_RELINK_ARGS); break;
        default: return hipErrorInvalidValue;
    }
#undef GP_RELINK_ARGS
    return hipGetLastError();
}

// next'/prev' of a run larger than the last-level cache go out as streaming
// stores: they would not stay cached for the kernels that read them, and the
// cache keeps what those kernels reuse (the run's size from its label tiles,
// at most a tile per mesh over).  Smaller runs keep them cached.
template <bool CM>
hipError_t launch_relink(const LaunchCfg &cfg, const RunBuffers &rb, hipStream_t s, size_t lds, int cmp_tb) {
    const bool stream_out = 24ll * rb.tri_tiles * cfg.block_label * cfg.items_label > kStreamOutBytes;
    return stream_out ? launch_relink_nt<CM, true>(cfg, rb, s, lds, cmp_tb)
                      : launch_relink_nt<CM, false>(cfg, rb, s, lds, cmp_tb);
}

bool small_fits(const LaunchCfg &cfg, int max_nt) {
    return max_nt >= 0 && max_nt <= cfg.small_max && max_nt <= kSmallMaxTri &&
           small_lds_bytes(max_nt) <= (size_t)cfg.lds_max;
}

bool runs_small(const LaunchCfg &cfg, const RunBuffers &rb) { return !rb.chain_only && small_fits(cfg, rb.max_nt); }

hipError_t launch_small_one(const MeshDesc &d, MeshCounters *host, hipStream_t s) {
    const dim3 grid(1), block(kSmallBlock);
    const size_t lds = small_lds_bytes(d.nt);
    if (d.nt <= kSmallBlock)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_small_one<3>), grid, block, lds, s, d, host);
    else if (d.nt <= 2 * kSmallBlock)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_small_one<6>), grid, block, lds, s, d, host);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_small_one<12>), grid, block, lds, s, d, host);
    return hipGetLastError();
}

int prepare_small(int lds_block) {
    const void *const fns[9] = {reinterpret_cast<const void *>(&k_small<3>),
                                reinterpret_cast<const void *>(&k_small<6>),
                                reinterpret_cast<const void *>(&k_small<12>),
                                reinterpret_cast<const void *>(&k_small_one<3>),
                                reinterpret_cast<const void *>(&k_small_one<6>),
                                reinterpret_cast<const void *>(&k_small_one<12>),
                                reinterpret_cast<const void *>(&k_small_jobs<3>),
                                reinterpret_cast<const void *>(&k_small_jobs<6>),
                                reinterpret_cast<const void *>(&k_small_jobs<12>)};
    int fixed = 0;
    for (const void *f : fns) {
        hipFuncAttributes a{};
        if (hipFuncGetAttributes(&a, f) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        fixed = (int)a.sharedSizeBytes > fixed ? (int)a.sharedSizeBytes : fixed;
    }
    const int dyn = lds_block - fixed;
    if (dyn <= 0) return 0;
    if (dyn > 65536 - fixed)
        for (const void *f : fns)
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess) {
                (void)hipGetLastError();
                return 65536 - fixed;
            }
    return dyn;
}

hipError_t launch_pipeline(const LaunchCfg &cfg, const RunBuffers &rb, hipStream_t s, launch_hook hook,
                           void *user) {
    auto H = [&](int k, int after) {
        if (hook) hook(user, k, after);
    };
    if (rb.nmesh <= 0) return hipSuccess;
    if (runs_small(cfg, rb)) {   // every mesh fits one workgroup: one launch
        const dim3 grid(rb.nmesh), block(kSmallBlock);
        const size_t lds = small_lds_bytes(rb.max_nt);
        H(K_SMALL, 0);
        if (rb.max_nt <= kSmallBlock)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_small<3>), grid, block, lds, s, rb.descs);
        else if (rb.max_nt <= 2 * kSmallBlock)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_small<6>), grid, block, lds, s, rb.descs);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_small<12>), grid, block, lds, s, rb.descs);
        H(K_SMALL, 1);
        return hipGetLastError();
    }
    const int pb = cfg.persistent_blocks, pt = cfg.block_persistent;
    const int cmp_tb = cfg.block_compact * cfg.items_compact;   // triangles per compaction tile

    H(K_LABEL, 0);
    {
        const ClearArgs ca = {rb.rc, rb.ctrs, rb.status, rb.cmp_tiles, rb.walk_counts, rb.emit_counts,
                              rb.wbuf_counts};
        GP_LAUNCH_ITEMS(k_label, cfg.items_label, dim3(rb.tri_tiles), dim3(cfg.block_label),
                        sizeof(int) * 3 * (size_t)cfg.block_label * cfg.items_label, s, rb.descs, rb.nmesh, ca);
    }
    H(K_LABEL, 1);

    H(K_RELINK, 0);
    {
        const size_t lds = (sizeof(int) * 3 + 2 + 4 + 1) * (size_t)cfg.block_relink * cfg.items_relink;
        const hipError_t e = rb.compact ? launch_relink<true>(cfg, rb, s, lds, cmp_tb)
                                        : launch_relink<false>(cfg, rb, s, lds, cmp_tb);
        if (e != hipSuccess) return e;
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
    hipLaunchKernelGGL((k_walk<kWalkItems, kWalkBuf>), dim3(pb), dim3(256), 0, s, rb.descs, rb.walk,
                       rb.walk_counts, rb.walk_cap, rb.status, cmp_tb, rb.wbuf, rb.wbuf_counts, rb.wbuf_cap);
    H(K_WALK, 1);

    H(K_TSCAN, 0);
    hipLaunchKernelGGL(k_tile_scan, dim3(rb.nmesh, rb.max_chunks), dim3(1024), 0, s, rb.descs, rb.status,
                       rb.cpre, cmp_tb);
    H(K_TSCAN, 1);

    H(K_COMPACT, 0);
    GP_LAUNCH_ITEMS(k_compact, cfg.items_compact, dim3(rb.cmp_tiles), dim3(cfg.block_compact),
                    compact_lds_bytes(cmp_tb), s, rb.descs, rb.nmesh,
                    rb.status, rb.cpre, rb.emit, rb.emit_counts, rb.emit_cap, rb.wbuf);
    H(K_COMPACT, 1);

    H(K_EMIT, 0);
    hipLaunchKernelGGL(k_emit<4>, dim3(pb), dim3(256), 0, s, rb.descs, rb.emit, rb.emit_counts, rb.emit_cap);
    H(K_EMIT, 1);
    return hipGetLastError();
}

}  // namespace gp
