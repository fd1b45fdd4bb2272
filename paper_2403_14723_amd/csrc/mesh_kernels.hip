// Polylla pipeline kernels for gfx950 (wave64).
//
// One run processes a batch of meshes through a per-mesh descriptor table
// (a plain call is a batch of one).  Streaming kernels tile each mesh
// separately, so a workgroup never straddles two meshes and all indices it
// handles are local to one mesh; data-dependent work (tips, repair seeds,
// fix-ups) goes through small device lists read by persistent grids.
//
// Kernel chain (paper Section 6, Algorithm 7, restructured):
//   k_init     clears run counters, per-mesh counters and scan tile status
//   k_label    longest edge per triangle (Section 6.1, Algorithm 8)
//   k_relink   frontier test (Section 6.2, Algorithm 9), terminal-edge seeds
//              (Section 6.3, Algorithm 10) and next/prev of every frontier
//              half-edge by turning around its target / origin (Section 6.5,
//              Algorithm 12); records barrier tips
//   k_repair   middle edge at each barrier tip (Section 6.4, Algorithm 11)
//   k_fixup    recomputes next/prev around the endpoints of new frontier edges
//   k_walk     from every seed: move to a frontier half-edge (Section 6.5.1,
//              Algorithm 13), walk its loop, record minimum and length at the
//              minimum's triangle (Section 6.6, Algorithm 14)
//   k_walk_rep the same for the seeds made by the repair
//   k_compact  scan of loop minima and lengths with decoupled look-back,
//              writing seeds, loop offsets and the loops themselves
//              (Section 6.7)
#include "gp_internal.h"

namespace gp {

const char *const kKernelNames[K_COUNT] = {"k_init", "k_label", "k_relink", "k_repair",
                                           "k_fixup", "k_walk", "k_compact"};

// ---------------------------------------------------------------------------
// half-edge queries (implicit triangle layout, Section 4.2)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int he_next(int h) {
    int t = h / 3;
    return (h - 3 * t == 2) ? h - 2 : h + 1;
}
__device__ __forceinline__ int he_prev(int h) {
    int t = h / 3;
    return (h - 3 * t == 0) ? h + 2 : h - 1;
}

__device__ __forceinline__ long long sq_len(int2 a, int2 b) {
    long long dx = (long long)b.x - a.x, dy = (long long)b.y - a.y;
    return dx * dx + dy * dy;
}

// Frontier test after the repair: boundary, longest edge of neither side, or
// added by the repair.  Before the repair the repair bits are all zero.
__device__ __forceinline__ bool is_frontier(const int32_t *__restrict__ twin,
                                            const uint8_t *__restrict__ tflag, int h) {
    int t = h / 3, i = h - 3 * t;
    uint32_t f = tflag[t];
    if ((f >> (2 + i)) & 1u) return true;
    int g = twin[h];
    if (g < 0) return true;
    if ((int)(f & 3u) == i) return false;
    int tg = g / 3;
    return (int)(tflag[tg] & 3u) != g - 3 * tg;
}

// next'(h): first frontier half-edge met turning clockwise around target(h),
// starting from next(h).  Returns -1 if the guard trips.
__device__ __forceinline__ int turn_next(const int32_t *__restrict__ twin,
                                         const uint8_t *__restrict__ tflag, int h) {
    int n = he_next(h);
    for (int k = 0; k < kRotGuard; k++) {
        if (is_frontier(twin, tflag, n)) return n;
        int g = twin[n];
        if (g < 0) return -1;
        n = he_next(g);
    }
    return -1;
}

// prev'(h): the mirror turn around origin(h), starting from prev(h).
__device__ __forceinline__ int turn_prev(const int32_t *__restrict__ twin,
                                         const uint8_t *__restrict__ tflag, int h) {
    int p = he_prev(h);
    for (int k = 0; k < kRotGuard; k++) {
        if (is_frontier(twin, tflag, p)) return p;
        int g = twin[p];
        if (g < 0) return -1;
        p = he_prev(g);
    }
    return -1;
}

// ---------------------------------------------------------------------------
// wave / block helpers
// ---------------------------------------------------------------------------

// Appends one entry per lane with pred set; one atomic per wave.  Must be
// reached by every active lane of the wave.
__device__ __forceinline__ int wave_reserve(int32_t *counter, bool pred) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return -1;
    int lane = __lane_id();
    int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(mask));
    base = __shfl(base, leader);
    return pred ? base + __popcll(mask & ((1ull << lane) - 1ull)) : -1;
}

__device__ __forceinline__ void wave_incl_scan2(int &a, int &b) {
    int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int ta = __shfl_up(a, d), tb = __shfl_up(b, d);
        if (lane >= d) {
            a += ta;
            b += tb;
        }
    }
}

// Exclusive block scan of a pair; lds must hold 3*16 ints per component.
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

// ---------------------------------------------------------------------------
// k_init
// ---------------------------------------------------------------------------

__global__ void k_init(RunCounters *rc, MeshCounters *ctrs, int nmesh, uint64_t *status,
                       int nstatus) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int stride = gridDim.x * blockDim.x;
    if (i == 0) {
        rc->ntips = 0;
        rc->ncand = 0;
        rc->nfix = 0;
        rc->tile_ctr = 0;
        rc->err = 0;
    }
    for (int k = i; k < nmesh; k += stride) {
        MeshCounters z = {};
        ctrs[k] = z;
    }
    for (int k = i; k < nstatus; k += stride) status[k] = 0ull;
}

// ---------------------------------------------------------------------------
// k_label: longest edge of each triangle
// ---------------------------------------------------------------------------

template <int ITEMS>
__global__ void k_label(const MeshDesc *__restrict__ descs, int nmesh) {
    const int tile = blockIdx.x;
    const int mi = find_mesh<0>(descs, nmesh, tile);
    const MeshDesc &d = descs[mi];
    const int nt = d.nt;
    const int base = (tile - d.tri_tile0) * (int)blockDim.x * ITEMS;
    const int32_t *__restrict__ org = d.org;
    const int2 *__restrict__ xy = d.xy;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        int t = base + j * (int)blockDim.x + (int)threadIdx.x;
        if (t >= nt) break;
        int2 p0 = xy[org[3 * t]], p1 = xy[org[3 * t + 1]], p2 = xy[org[3 * t + 2]];
        long long l0 = sq_len(p0, p1), l1 = sq_len(p1, p2), l2 = sq_len(p2, p0);
        long long m = l0 > l1 ? l0 : l1;
        m = m > l2 ? m : l2;
        int cnt = (l0 == m) + (l1 == m) + (l2 == m);
        int best;
        if (cnt == 1) {
            best = l0 == m ? 0 : (l1 == m ? 1 : 2);
        } else {
            // tie at the maximum: the lower edge id min(h, twin h) wins
            best = -1;
            int bid = 0x7fffffff;
            long long ls[3] = {l0, l1, l2};
            for (int i = 0; i < 3; i++) {
                if (ls[i] != m) continue;
                int h = 3 * t + i, g = d.twin[h];
                int id = (g >= 0 && g < h) ? g : h;
                if (id < bid) {
                    bid = id;
                    best = i;
                }
            }
            atomicAdd(&d.ctr->nties, 1);
        }
        d.tflag[t] = (uint8_t)best;
        d.pl[t] = 0;
    }
}

// ---------------------------------------------------------------------------
// k_relink: frontier labels, seeds, next/prev, barrier tips
// ---------------------------------------------------------------------------

constexpr uint32_t kSeedBit = 1u << 5;   // tflag: the longest edge of t is a terminal seed

template <int ITEMS>
__global__ void k_relink(const MeshDesc *__restrict__ descs, int nmesh, RunCounters *rc,
                         ListEntry *tips, int cap_tips) {
    const int tile = blockIdx.x;
    const int mi = find_mesh<1>(descs, nmesh, tile);
    const MeshDesc &d = descs[mi];
    const int nh = 3 * d.nt;
    const int base = (tile - d.he_tile0) * (int)blockDim.x * ITEMS;
    const int32_t *__restrict__ twin = d.twin;
    uint8_t *__restrict__ tflag = d.tflag;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        int h = base + j * (int)blockDim.x + (int)threadIdx.x;
        bool tip = false;
        bool err = false;
        if (h < nh) {
            int t = h / 3, i = h - 3 * t;
            uint32_t f = tflag[t];
            int L = (int)(f & 3u);
            int g = twin[h];
            bool g_long = false;
            if (g >= 0) {
                int tg = g / 3;
                g_long = (int)(tflag[tg] & 3u) == g - 3 * tg;
            }
            bool F = g < 0 || (L != i && !g_long);
            int n = -1, p = -1;
            if (F) {
                n = turn_next(twin, tflag, h);
                p = turn_prev(twin, tflag, h);
                err = n < 0 || p < 0;
                tip = g >= 0 && n == g;
            }
            d.next_o[h] = n;
            d.prev_o[h] = p;
            // terminal edge: longest on both sides (the lower half-edge is the
            // seed), or longest and on the boundary
            if (L == i && (g < 0 || (g_long && h < g))) tflag[t] = (uint8_t)(f | kSeedBit);
        }
        int slot = wave_reserve(&rc->ntips, tip);
        if (tip) {
            if (slot < cap_tips) {
                tips[slot].mesh = mi;
                tips[slot].he = h;
                atomicAdd(&d.ctr->ntips, 1);
            } else {
                err = true;
            }
        }
        if (err) atomicOr(&d.ctr->err, kErrCorrupt);
    }
}

// ---------------------------------------------------------------------------
// k_repair: middle edge of each barrier tip
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t set_repair_bit(uint8_t *tflag, int h) {
    int t = h / 3, i = h - 3 * t;
    uint32_t *word = reinterpret_cast<uint32_t *>(tflag) + (t >> 2);
    uint32_t bit = (1u << (2 + i)) << (8 * (t & 3));
    return atomicOr(word, bit) & bit;
}

__global__ void k_repair(const MeshDesc *__restrict__ descs, RunCounters *rc, const ListEntry *tips,
                         int cap_tips, ListEntry *cands, int cap_cands, ListEntry *fixes, int cap_fix) {
    const int ntips = min(rc->ntips, cap_tips);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ntips; k += gridDim.x * blockDim.x) {
        const ListEntry e = tips[k];
        const MeshDesc &d = descs[e.mesh];
        const int32_t *__restrict__ twin = d.twin;
        // a: the only frontier edge at the tip v = target(e.he), leaving v
        const int a = twin[e.he];
        bool err = a < 0;
        int deg = 0, r = a;
        while (!err) {   // degree: a full clockwise turn around v
            int g = twin[r];
            if (g < 0 || ++deg > kRotGuard) {
                err = true;
                break;
            }
            r = he_next(g);
            if (r == a) break;
        }
        if (err) {
            atomicOr(&d.ctr->err, kErrCorrupt);
            continue;
        }
        int m = a;
        for (int s = 0; s < deg / 2; s++) m = he_next(twin[m]);
        const int mt = twin[m];
        uint32_t had_lo = set_repair_bit(d.tflag, m < mt ? m : mt);
        set_repair_bit(d.tflag, m < mt ? mt : m);
        if (!had_lo) atomicAdd(&d.ctr->nmiddle, 1);
        int c = atomicAdd(&rc->ncand, 2);
        if (c + 1 < cap_cands) {
            cands[c].mesh = e.mesh;
            cands[c].he = m;
            cands[c + 1].mesh = e.mesh;
            cands[c + 1].he = mt;
        } else {
            atomicOr(&d.ctr->err, kErrCorrupt);
        }
        int f = atomicAdd(&rc->nfix, 2);
        if (f + 1 < cap_fix) {
            fixes[f].mesh = e.mesh;
            fixes[f].he = a;      // leaves the tip
            fixes[f + 1].mesh = e.mesh;
            fixes[f + 1].he = mt; // leaves the other endpoint of the middle edge
        } else {
            atomicOr(&d.ctr->err, kErrCorrupt);
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
    int p = he_prev(e);
    bool ok = true;
    if (is_frontier(twin, tflag, p)) {
        int n = turn_next(twin, tflag, p);
        ok &= n >= 0;
        d.next_o[p] = n;
    }
    if (is_frontier(twin, tflag, e)) {
        int q = turn_prev(twin, tflag, e);
        ok &= q >= 0;
        d.prev_o[e] = q;
    }
    return ok;
}

__global__ void k_fixup(const MeshDesc *__restrict__ descs, RunCounters *rc, const ListEntry *fixes,
                        int cap_fix) {
    const int nfix = min(rc->nfix, cap_fix);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nfix; k += gridDim.x * blockDim.x) {
        const ListEntry en = fixes[k];
        const MeshDesc &d = descs[en.mesh];
        const int32_t *__restrict__ twin = d.twin;
        const int o = en.he;
        bool ok = true, open = false;
        int e = o, steps = 0;
        do {   // clockwise over the outgoing half-edges
            ok &= fix_around(d, e);
            int g = twin[e];
            if (g < 0) {
                open = true;
                break;
            }
            e = he_next(g);
            if (++steps > kRotGuard) {
                ok = false;
                break;
            }
        } while (e != o);
        if (open && ok) {   // a boundary vertex: also go counter-clockwise
            e = o;
            steps = 0;
            while (true) {
                int g = twin[he_prev(e)];
                if (g < 0) break;
                e = g;
                ok &= fix_around(d, e);
                if (++steps > kRotGuard) {
                    ok = false;
                    break;
                }
            }
        }
        if (!ok) atomicOr(&d.ctr->err, kErrCorrupt);
    }
}

// ---------------------------------------------------------------------------
// k_walk: seed -> frontier half-edge -> loop minimum and length
// ---------------------------------------------------------------------------

// Walks the loop through frontier half-edge f; records (length, local index
// of the minimum) in the minimum's triangle.  All seeds of one loop write the
// same byte.
__device__ __forceinline__ bool walk_record(const MeshDesc &d, int f) {
    const int32_t *__restrict__ nx = d.next_o;
    const int nh = 3 * d.nt;
    int cur = f, mn = f, len = 0;
    do {
        mn = cur < mn ? cur : mn;
        ++len;
        cur = nx[cur];
        if (cur < 0 || len > nh) return false;
    } while (cur != f);
    int t = mn / 3;
    int code = ((len < kPlMax ? len : kPlMax) << 2) | (mn - 3 * t);
    d.pl[t] = (uint8_t)code;
    return true;
}

// From seed s, turn clockwise around origin(s) until a frontier half-edge.
// After the fix-up, next_o[h] >= 0 exactly on frontier half-edges.
__device__ __forceinline__ int seek_frontier(const MeshDesc &d, int s) {
    const int32_t *__restrict__ nx = d.next_o;
    int f = s;
    for (int k = 0; k < kRotGuard; k++) {
        if (nx[f] >= 0) return f;
        int g = d.twin[f];
        if (g < 0) return -1;
        f = he_next(g);
    }
    return -1;
}

template <int ITEMS>
__global__ void k_walk(const MeshDesc *__restrict__ descs, int nmesh) {
    const int tile = blockIdx.x;
    const int mi = find_mesh<0>(descs, nmesh, tile);
    const MeshDesc &d = descs[mi];
    const int nt = d.nt;
    const int base = (tile - d.tri_tile0) * (int)blockDim.x * ITEMS;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        int t = base + j * (int)blockDim.x + (int)threadIdx.x;
        if (t >= nt) break;
        uint32_t f = d.tflag[t];
        if (!(f & kSeedBit)) continue;
        int L = (int)(f & 3u);
        // the seed triangle lies in the polygon; any of its frontier
        // half-edges is on the polygon's loop
        int s = -1;
        for (int i = 1; i <= 3 && s < 0; i++) {
            int h = 3 * t + (L + i) % 3;
            if (d.next_o[h] >= 0) s = h;
        }
        if (s < 0) s = seek_frontier(d, 3 * t + L);
        if (s < 0 || !walk_record(d, s)) atomicOr(&d.ctr->err, kErrCorrupt);
    }
}

__global__ void k_walk_rep(const MeshDesc *__restrict__ descs, RunCounters *rc,
                           const ListEntry *cands, int cap_cands) {
    const int n = min(rc->ncand, cap_cands);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const ListEntry e = cands[k];
        const MeshDesc &d = descs[e.mesh];
        int s = seek_frontier(d, e.he);
        if (s < 0 || !walk_record(d, s)) atomicOr(&d.ctr->err, kErrCorrupt);
    }
}

// ---------------------------------------------------------------------------
// k_compact: decoupled look-back scan of (loop count, loop length) per mesh,
// then each loop is written starting at its minimum
// ---------------------------------------------------------------------------

constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr int kSpinGuard = 1 << 26;

__device__ __forceinline__ uint64_t pack_status(uint64_t flag, int cnt, int sum) {
    return flag | ((uint64_t)(uint32_t)cnt << 32 & 0x3fffffff00000000ull) | (uint32_t)sum;
}

// Length of the loop starting at its minimum mn (used when it did not fit in
// the per-triangle byte).
__device__ __forceinline__ int loop_length(const MeshDesc &d, int mn) {
    const int nh = 3 * d.nt;
    int cur = mn, len = 0;
    do {
        ++len;
        cur = d.next_o[cur];
        if (cur < 0 || len > nh) return -1;
    } while (cur != mn);
    return len;
}

template <int ITEMS>
__global__ void k_compact(const MeshDesc *__restrict__ descs, int nmesh, RunCounters *rc,
                          uint64_t *status) {
    __shared__ int s_tile;
    __shared__ int lds[80];
    __shared__ int s_prefix[2];
    if (threadIdx.x == 0) s_tile = atomicAdd(&rc->tile_ctr, 1);
    __syncthreads();
    const int tile = s_tile;
    const int mi = find_mesh<2>(descs, nmesh, tile);
    const MeshDesc &d = descs[mi];
    const int nt = d.nt;
    const int ltile = tile - d.cmp_tile0;
    const int per_tile = (int)blockDim.x * ITEMS;
    const int mesh_tiles = nt > 0 ? (nt + per_tile - 1) / per_tile : 1;
    const int t0 = ltile * per_tile + (int)threadIdx.x * ITEMS;

    // 1. this thread's loop minima and lengths (contiguous triangles)
    uint8_t code[ITEMS];
    int lens[ITEMS];
    int cnt = 0, sum = 0;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        int t = t0 + j;
        code[j] = t < nt ? d.pl[t] : 0;
        lens[j] = 0;
        if (code[j]) {
            int len = code[j] >> 2;
            if (len >= kPlMax) len = loop_length(d, 3 * t + (code[j] & 3));
            if (len < 0) {
                bad = true;
                len = 0;
            }
            lens[j] = len;
            cnt += 1;
            sum += len;
        }
    }
    // 2. block scan
    int ecnt, esum, tcnt, tsum;
    block_excl_scan2(cnt, sum, ecnt, esum, tcnt, tsum, lds);
    // 3. look-back over the tiles of the same mesh
    if (threadIdx.x == 0) {
        int pc = 0, ps = 0;
        if (ltile == 0) {
            __hip_atomic_store(&status[tile], pack_status(kFlagInc, tcnt, tsum), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&status[tile], pack_status(kFlagAgg, tcnt, tsum), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            int k = tile - 1;
            int spins = 0;
            while (true) {
                uint64_t st = __hip_atomic_load(&status[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                uint64_t flag = st & (3ull << 62);
                if (flag == 0ull) {
                    if (++spins > kSpinGuard) {
                        atomicOr(&d.ctr->err, kErrCorrupt);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                pc += (int)((st >> 32) & 0x3fffffffull);
                ps += (int)(uint32_t)st;
                if (flag == kFlagInc || k == d.cmp_tile0) break;
                --k;
            }
            __hip_atomic_store(&status[tile], pack_status(kFlagInc, pc + tcnt, ps + tsum),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_prefix[0] = pc;
        s_prefix[1] = ps;
        if (ltile == mesh_tiles - 1) {
            d.ctr->npoly = pc + tcnt;
            d.ctr->nloop = ps + tsum;
            d.loop_off[pc + tcnt] = ps + tsum;
        }
    }
    __syncthreads();
    // 4. emit seeds, offsets and loops
    const int nh = 3 * nt;
    int p = s_prefix[0] + ecnt, off = s_prefix[1] + esum;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        if (!code[j]) continue;
        int t = t0 + j;
        int mn = 3 * t + (code[j] & 3);
        if (p >= nt || off + lens[j] > nh) {  // only reachable with corrupt lengths
            bad = true;
            break;
        }
        d.seeds[p] = mn;
        d.loop_off[p] = off;
        int cur = mn;
        for (int k = 0; k < lens[j] && cur >= 0; k++) {
            d.loop_he[off + k] = cur;
            cur = d.next_o[cur];
        }
        if (cur != mn) bad = true;
        ++p;
        off += lens[j];
    }
    if (bad) atomicOr(&d.ctr->err, kErrCorrupt);
}

// ---------------------------------------------------------------------------
// host launch of the whole chain
// ---------------------------------------------------------------------------

#define GP_LAUNCH_ITEMS(KER, ITEMS_RT, GRID, BLOCK, STREAM, ...)                                 \
    do {                                                                                      \
        switch (ITEMS_RT) {                                                                   \
            case 1: hipLaunchKernelGGL(KER<1>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break;  \
            case 2: hipLaunchKernelGGL(KER<2>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break;  \
            case 4: hipLaunchKernelGGL(KER<4>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break;  \
            case 8: hipLaunchKernelGGL(KER<8>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break;  \
            default: return hipErrorInvalidValue;                                             \
        }                                                                                     \
    } while (0)

hipError_t launch_pipeline(const LaunchCfg &cfg, const RunBuffers &rb, hipStream_t s,
                           launch_hook hook, void *user) {
    auto H = [&](int k, int after) {
        if (hook) hook(user, k, after);
    };
    if (rb.nmesh <= 0) return hipSuccess;
    const int pb = cfg.persistent_blocks, pt = cfg.block_persistent;

    H(K_INIT, 0);
    {
        int n = rb.cmp_tiles > rb.nmesh ? rb.cmp_tiles : rb.nmesh;
        int grid = (n + 255) / 256;
        grid = grid < 1 ? 1 : (grid > 1024 ? 1024 : grid);
        hipLaunchKernelGGL(k_init, dim3(grid), dim3(256), 0, s, rb.rc, rb.ctrs, rb.nmesh, rb.status,
                           rb.cmp_tiles);
    }
    H(K_INIT, 1);

    H(K_LABEL, 0);
    if (rb.tri_tiles > 0)
        GP_LAUNCH_ITEMS(k_label, cfg.items_label, dim3(rb.tri_tiles), dim3(cfg.block_label), s,
                        rb.descs, rb.nmesh);
    H(K_LABEL, 1);

    H(K_RELINK, 0);
    if (rb.he_tiles > 0)
        GP_LAUNCH_ITEMS(k_relink, cfg.items_relink, dim3(rb.he_tiles), dim3(cfg.block_relink), s,
                        rb.descs, rb.nmesh, rb.rc, rb.tips, rb.cap_tips);
    H(K_RELINK, 1);

    H(K_REPAIR, 0);
    hipLaunchKernelGGL(k_repair, dim3(pb), dim3(pt), 0, s, rb.descs, rb.rc, rb.tips, rb.cap_tips,
                       rb.cands, rb.cap_cands, rb.fixes, rb.cap_fix);
    H(K_REPAIR, 1);

    H(K_FIXUP, 0);
    hipLaunchKernelGGL(k_fixup, dim3(pb), dim3(pt), 0, s, rb.descs, rb.rc, rb.fixes, rb.cap_fix);
    H(K_FIXUP, 1);

    H(K_WALK, 0);
    if (rb.tri_tiles > 0)
        GP_LAUNCH_ITEMS(k_walk, cfg.items_label, dim3(rb.tri_tiles), dim3(cfg.block_label), s,
                        rb.descs, rb.nmesh);
    hipLaunchKernelGGL(k_walk_rep, dim3(pb), dim3(pt), 0, s, rb.descs, rb.rc, rb.cands, rb.cap_cands);
    H(K_WALK, 1);

    H(K_COMPACT, 0);
    if (rb.cmp_tiles > 0)
        GP_LAUNCH_ITEMS(k_compact, cfg.items_compact, dim3(rb.cmp_tiles), dim3(cfg.block_compact), s,
                        rb.descs, rb.nmesh, rb.rc, rb.status);
    H(K_COMPACT, 1);
    return hipGetLastError();
}

}  // namespace gp
