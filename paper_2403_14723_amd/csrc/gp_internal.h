// Internal types shared by the gpolylla kernels and the host runtime.
//
// Device data layout (one mesh; all int32 unless noted; h = 3t+i):
//   xy[2V]      interleaved coordinates, read as int2 (one 8-byte gather)
//   org[3T]     origin vertex of each half-edge (counter-clockwise corners)
//   twin[3T]    opposite half-edge, -1 on the boundary
//   tflag[T]    uint8 per triangle: bits 0-1 local index of the longest edge,
//               bits 2-4 frontier bit of local edges 0..2, bit 5 seed
//   pl[T]       uint8 per triangle: 0, or (min(L,63) << 2 | i) when half-edge
//               3t+i is the minimum of a loop of length L
//   next_o/prev_o[3T], seeds[<=T], loop_off[<=T+1], loop_he[<=3T] (outputs)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gp {

constexpr int kWave = 64;
constexpr int kPlMax = 63;            // loop lengths >= 63: k_walk keeps them in lpos
constexpr int kRotGuard = 1 << 20;    // bound on turns around one vertex

// error bits collected on the device
constexpr int kErrCorrupt = 1;

// per-mesh counters, written by the kernels and read back once per run
struct MeshCounters {
    int32_t err;
    int32_t nterm;
    int32_t ntips;
    int32_t nmiddle;
    int32_t nties;
    int32_t npoly;
    int32_t nloop;
    int32_t chunks_done;   // k_tile_scan blocks finished (the last one scans the chunk totals)
};

// list sizes and the dynamic tile counter of one run
struct RunCounters {
    int32_t ntips;
    int32_t unused;
    int32_t nfix;
    int32_t tile_ctr;
    int32_t err;
    int32_t pad[3];
};

struct MeshDesc {
    const int2 *xy;
    const int32_t *org;
    const int32_t *twin;
    int32_t *next_o;
    int32_t *prev_o;
    uint8_t *tflag;
    uint8_t *pl;
    int32_t *seeds;
    int32_t *loop_off;
    int32_t *loop_he;
    int32_t *lpos;       // per triangle: where k_walk stored the loop whose minimum it holds
                         // (or that loop's length, when it is kPlMax or longer)
    MeshCounters *ctr;
    int32_t nt;
    int32_t nv;
    int32_t tri_tile0;   // first tile of this mesh in the triangle tile space
    int32_t he_tile0;    // first tile of this mesh in the relink tile space (triangles)
    int32_t cmp_tile0;   // first tile of this mesh in the compaction tile space
    int32_t esc_mask;    // compact meshes: escape table slots - 1
    // compact meshes (org and twin are null): per triangle {v0, (v1 - v0) |
    // (v2 - v0) << 16} and per half-edge twin - h as int16 (0: boundary);
    // a 16-bit field holding kEsc16 is in the escape table
    const int2 *org8;
    const int16_t *twin16;
    const int32_t *esc;  // (key, value) pairs: key h for a twin, ~h for corner h
};

static_assert(sizeof(MeshDesc) % 4 == 0, "descriptor tables are copied in 4-byte words");

struct ListEntry {
    int32_t mesh;
    int32_t he;
};

// a loop whose half-edges k_emit writes: minimum mn, first output slot off
struct EmitEntry {
    int32_t mesh;
    int32_t mn;
    int32_t off;
};

// Lists appended to by many workgroups are split into kStripes stripes, each
// with its own counter, so appends do not all hit one address.  Stripe s
// holds entries [s*cap, s*cap + min(count[s], cap)).
constexpr int kStripes = 64;
constexpr int kStripePad = 32;   // counters 128 bytes apart: one cache line each

// ---- launch plumbing (host side, defined in mesh_kernels.hip) ------------

// k_small: a mesh of at most kSmallMaxTri triangles can run as one workgroup
// of kSmallBlock threads with every intermediate array in LDS
constexpr int kSmallMaxTri = 4096;
constexpr int kSmallBlock = 1024;
// LDS of k_small for a mesh of nt triangles: per triangle four slots (one
// unused) of two 16-bit arrays and a 32-bit one, and a label byte
__host__ __device__ inline size_t small_a16_bytes(int nt) { return (8 * (size_t)nt + 15) / 16 * 16; }
__host__ __device__ inline size_t small_lab_bytes(int nt) { return ((size_t)nt + 15) / 16 * 16; }
inline size_t small_lds_bytes(int nt) { return 4 * small_a16_bytes(nt) + small_lab_bytes(nt); }

struct LaunchCfg {
    int block_label = 128, items_label = 4;
    int block_relink = 256, items_relink = 2;     // k_relink (tile <= 1024 triangles)
    int block_compact = 128, items_compact = 4;   // tile <= 2048 triangles (LDS 19 B each)
    int persistent_blocks = 2048;
    int block_persistent = 256;
    int small_max = kSmallMaxTri;   // k_small for batches whose meshes all have at most this many triangles
    int lds_max = 0;                // dynamic LDS bytes k_small may use on the device
};

struct RunBuffers {
    const MeshDesc *descs;   // device, nmesh entries
    int nmesh;
    bool compact;            // some mesh is in the compact encoding
    int32_t tri_tiles;       // total triangle tiles (label)
    int32_t he_tiles;        // total relink tiles
    int32_t cmp_tiles;       // total compaction tiles
    RunCounters *rc;         // device
    ListEntry *tips;         // capacity cap_tips
    ListEntry *fixes;        // capacity cap_fix
    int32_t cap_tips, cap_fix;
    uint64_t *status;        // per compaction tile: (loops << 32 | half-edges), then its prefix within its chunk
    uint64_t *cpre;          // per compaction tile; at each chunk's first tile: the chunk's prefix
    int32_t max_chunks;      // most chunks (of kScanChunk tiles) in one mesh
    MeshCounters *ctrs;      // device, nmesh entries
    ListEntry *walk;         // striped: seeds left open by k_relink and repair seeds
    int32_t *walk_counts;    // kStripes counters, kStripePad ints apart
    int32_t walk_cap;        // per stripe
    EmitEntry *emit;         // striped: loops k_compact leaves to k_emit
    int32_t *emit_counts;    // kStripes counters, kStripePad ints apart
    int32_t emit_cap;        // per stripe
    int32_t *wbuf;           // striped: walked loops (rotation index, then half-edges)
    int32_t *wbuf_counts;    // kStripes counters, kStripePad ints apart
    int32_t wbuf_cap;        // ints per stripe
    int32_t max_nt;          // the largest mesh of the batch
    bool chain_only;         // run the tiled chain even where k_small could
};

// k_walk records each chain's half-edges in LDS, up to this many; longer
// loops are left to k_emit
constexpr int kWalkBuf = 16;
constexpr long long kStreamOutBytes = 256ll << 20;   // MI355X's last-level cache (Infinity Cache)
constexpr int kWalkItems = 1;   // chains per k_walk thread
constexpr int kTileScanItems = 4;                   // compaction tiles per k_tile_scan thread
constexpr int kScanChunk = 1024 * kTileScanItems;   // compaction tiles per k_tile_scan block
// k_compact's LDS holds up to this many loop half-edges per 4 triangles of
// its tile (2.75 per triangle; meshes average about 2 or fewer).  A tile
// with more writes its loops straight to global memory.  With one seed and
// one offset per triangle that is 19 bytes per triangle, so eight tiles of
// 1024 triangles share a CU's LDS.
constexpr int kCompactHe4 = 11;
__host__ __device__ inline int compact_he_cap(int tile) { return tile / 4 * kCompactHe4; }
inline size_t compact_lds_bytes(int tile) {
    return sizeof(int) * ((size_t)compact_he_cap(tile) + 2 * (size_t)tile);
}

enum KernelId { K_LABEL = 0, K_RELINK, K_REPAIR, K_FIXUP, K_WALK, K_TSCAN, K_COMPACT, K_EMIT, K_SMALL, K_COUNT };
extern const char *const kKernelNames[K_COUNT];

// Per-kernel hooks so the runtime can bracket launches with events.
typedef void (*launch_hook)(void *user, int kernel_id, int after);

hipError_t launch_pipeline(const LaunchCfg &cfg, const RunBuffers &rb, hipStream_t s,
                           launch_hook hook, void *user);
// Whether meshes of at most max_nt triangles fit k_small, and whether a run
// of rb goes through it (one launch) instead of the chain.
bool small_fits(const LaunchCfg &cfg, int max_nt);
bool runs_small(const LaunchCfg &cfg, const RunBuffers &rb);
// One small mesh on its own: its descriptor as a kernel argument (d.ctr may
// be null) and its counts written to coherent host memory.
hipError_t launch_small_one(const MeshDesc &d, MeshCounters *host, hipStream_t s);
// Lets k_small use the current device's LDS per workgroup (lds_block bytes,
// less its own static LDS); returns the dynamic LDS bytes it may then ask for
// (0: none).  Once per device, before its first launch.
int prepare_small(int lds_block);

// Copies `bytes` (a multiple of 4) with a kernel on stream s; either side may
// be coherent pinned host memory.
hipError_t launch_copy_words(void *dst, const void *src, size_t bytes, hipStream_t s);

// Writes one descriptor into device memory with a kernel (its value travels
// as a kernel argument), so no host staging buffer is needed.
hipError_t launch_put_desc(const MeshDesc &d, MeshDesc *dst, hipStream_t s);
// Writes the counts of mesh counters c as 8 int32: status (0 or -10), npoly,
// nloop, ntips, nmiddle, nties, 0, 0.
hipError_t launch_export_counts(const MeshCounters *c, int32_t *out, hipStream_t s);

// tiles of one mesh for a given tile size; every mesh has at least one tile
// so that an empty mesh still gets its loop_off[0] written
inline int32_t tiles_for(int64_t n, int64_t tile) {
    int64_t k = (n + tile - 1) / tile;
    return (int32_t)(k < 1 ? 1 : k);
}

// ---- small jobs: build and mesh in one workgroup (mesh_kernels.hip) -------
//
// A job of at most kJobSmallTri triangles and kJobSmallV vertices, its
// inputs already on the device: one workgroup checks and orients it, matches
// its twins in LDS, then meshes it as k_small does.  counts receives the
// mesh counters (kJobCounts ints: the 8 of MeshCounters, the build's error
// key as two words (~0 when the build passed), the triangles it flipped).
constexpr int kJobSmallTri = kSmallMaxTri;
constexpr int kJobSmallV = 4096;
constexpr int kJobCounts = 12;
struct SmallJob {
    const int2 *xy;
    const int32_t *tri;
    int32_t nv, nt;
    int32_t *org, *twin;   // 3 nt each: the built structure
    int32_t *next_o, *prev_o, *seeds, *loop_off, *loop_he;
    int32_t *counts;
    int2 *xy_out;          // when set, xy is copied here (the built mesh's own coordinates)
    int32_t build_only;    // 1: stop after the build (a mesh for later runs)
    int32_t pad;
};
// dynamic LDS of one such workgroup
size_t small_job_lds_bytes(int max_nv, int max_nt);
hipError_t launch_small_jobs(const SmallJob *jobs, int n, int max_nv, int max_nt, hipStream_t s);

// ---- build (build_kernels.hip) -------------------------------------------

struct BuildBuffers {
    const int2 *xy;
    const int32_t *tri;
    int32_t nv, nt;
    int32_t *org, *twin;
    int32_t *deg;      // nv + 1, zeroed by the build
    int32_t *vstart;   // nv + 1
    int32_t *fill;     // nv
    int2 *bucket;      // 3 nt: (half-edge, its target vertex), grouped by origin
    uint64_t *scan_status;  // scan tiles
    int32_t *scan_ctr;
    unsigned long long *err_key;  // lowest (rank << 8 | code) seen
    int32_t *nflipped;
};

hipError_t launch_build_orient(const BuildBuffers &b, hipStream_t s);
hipError_t launch_build_link(const BuildBuffers &b, hipStream_t s);
int32_t build_scan_tiles(int32_t n);

// ---- renumbering along a Z-order curve (renumber.hip) ---------------------

struct RenumberBuffers {
    const int2 *xy_in;
    const int32_t *tri_in;
    int32_t nv, nt;
    int2 *xy_out;          // nv, in the new vertex order
    int32_t *tri_out;      // 3 nt, new triangle order, new vertex indices
    int32_t *vperm;        // nv: new -> old vertex
    int32_t *tperm;        // nt: new -> old triangle
    int32_t *vinv;         // nv: old -> new vertex (scratch)
    uint64_t *keys, *keys_alt;   // max(nv, nt) each (scratch)
    int32_t *vals;               // max(nv, nt) (scratch)
    void *sort_tmp;              // sort_bytes (scratch)
    size_t sort_bytes;
};

// scratch bytes of the radix sort of n key-value pairs
size_t renumber_sort_bytes(int32_t n);
hipError_t launch_renumber(const RenumberBuffers &b, hipStream_t s);

// ---- compact half-edge encoding (build_kernels.hip) ----------------------
//
// A compact mesh keeps its corners and twins in 16-bit offsets: the twin of
// h as twin - h, the corners of a triangle as v0 plus v1 - v0 and v2 - v0.
// Values whose offset does not fit (or is 0 for a twin, which means
// boundary) are kept in an open-addressing hash table of (key, value) pairs:
// key h for the twin of h, ~h for corner h (the org of half-edge h).

constexpr int kEsc16 = -32768;               // the value is in the escape table
constexpr int32_t kEscEmpty = (int32_t)0x80000000u;   // an empty table slot

__host__ __device__ inline uint32_t esc_hash(int32_t key) {
    uint32_t x = (uint32_t)key * 0x9E3779B1u;
    return x ^ (x >> 15);
}

struct CompactBuffers {
    const int32_t *org, *twin;   // the int32 structure (input of the encoder)
    int32_t nt;
    int2 *org8;
    int16_t *twin16;
    int32_t *esc;                // 2 * (esc_mask + 1) ints
    int32_t esc_mask;
    int32_t *nesc;               // escapes counted by the encoder
};

// org8 and twin16, and the number of escapes into *nesc (zeroed by the caller)
hipError_t launch_compact_encode(const CompactBuffers &c, hipStream_t s);
// the escape table (cleared, then filled); needs esc and esc_mask
hipError_t launch_compact_escapes(const CompactBuffers &c, hipStream_t s);
// org and twin (int32) decoded from org8, twin16 and the table
hipError_t launch_compact_decode(const CompactBuffers &c, int32_t *org, int32_t *twin, hipStream_t s);

}  // namespace gp
