// Objects behind the opaque handles of include/gpolylla.h, shared by the
// runtime (runtime.cpp) and the serving loop (serve.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <unordered_map>
#include <vector>

#include "../../include/gpolylla.h"
#include "gp_internal.h"

namespace gprt {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t n, size_t a = kAlign) { return (n + a - 1) / a * a; }

// Device memory of one context.  Two modes:
//  - caching (default): blocks are kept after release and handed out again
//    for requests of up to 12.5% smaller size;
//  - arena: one block reserved up front, allocations bump through it,
//    release does nothing and reset() frees everything at once (the serving
//    loop resets a lane's arena when the lane's batch is done).
// All users of one pool run on one stream, so reuse after release (or after
// a reset) is ordered after earlier work by the stream.
class DevPool {
  public:
    size_t cap = 0;
    size_t held = 0;
    size_t in_use = 0;

    int make_arena(size_t bytes) {
        bytes = align_up(bytes);
        void *q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return GP_ENOMEM;
        }
        arena_ = static_cast<char *>(q);
        arena_cap_ = bytes;
        arena_off_ = 0;
        held = bytes;
        return GP_OK;
    }
    bool is_arena() const { return arena_ != nullptr; }
    size_t arena_free() const { return arena_cap_ - arena_off_; }
    void reset() {
        arena_off_ = 0;
        in_use = 0;
    }

    int alloc(size_t n, void **p) {
        n = align_up(n ? n : kAlign);
        if (arena_) {
            if (arena_off_ + n > arena_cap_) return GP_ENOMEM;
            *p = arena_ + arena_off_;
            arena_off_ += n;
            in_use += n;
            return GP_OK;
        }
        auto it = free_.lower_bound(n);
        if (it != free_.end() && it->first <= n + n / 8) {
            *p = it->second;
            in_use += it->first;
            used_[*p] = it->first;
            free_.erase(it);
            return GP_OK;
        }
        if (cap && held + n > cap) trim();
        if (cap && held + n > cap) return GP_ENOMEM;
        void *q = nullptr;
        if (hipMalloc(&q, n) != hipSuccess) {
            (void)hipGetLastError();
            trim();
            if (hipMalloc(&q, n) != hipSuccess) {
                (void)hipGetLastError();
                return GP_ENOMEM;
            }
        }
        held += n;
        in_use += n;
        used_[q] = n;
        *p = q;
        return GP_OK;
    }
    void release(void *p) {
        if (!p || arena_) return;
        auto it = used_.find(p);
        if (it == used_.end()) return;
        in_use -= it->second;
        free_.emplace(it->second, p);
        used_.erase(it);
    }
    void trim() {
        for (auto &kv : free_) {
            (void)hipFree(kv.second);
            held -= kv.first;
        }
        free_.clear();
    }
    void destroy() {
        trim();
        for (auto &kv : used_) (void)hipFree(kv.first);
        used_.clear();
        if (arena_) (void)hipFree(arena_);
        arena_ = nullptr;
        held = in_use = 0;
    }

  private:
    std::multimap<size_t, void *> free_;
    std::unordered_map<void *, size_t> used_;
    char *arena_ = nullptr;
    size_t arena_cap_ = 0, arena_off_ = 0;
};

// A bump arena carved out of one pool block.
struct Arena {
    char *base = nullptr;
    size_t size = 0, off = 0;
    template <class T>
    T *take(size_t count) {
        size_t n = align_up(count * sizeof(T));
        T *p = reinterpret_cast<T *>(base + off);
        off += n;
        return p;
    }
};

template <class T>
size_t arena_bytes(size_t count) {
    return align_up(count * sizeof(T));
}

struct RunState;
struct GraphCache;

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Builds n half-edge structures (the work of gpolylla_build_halfedges for
// each) with two host checks in all, on the context's stream: out[i] and
// status[i] per build.  Returns GP_ENOMEM when the host staging cannot be
// allocated (nothing built), else GP_OK.
// Coherent pinned host blocks cached per context (a block of at least n
// bytes, reused when it is at most twice that; give back with its size).
void *pinned_take(gp_ctx *c, size_t n);
void pinned_give(gp_ctx *c, void *p, size_t n);

int build_many(gp_ctx *c, int n, const int32_t *const *xy, const int32_t *nv, const int32_t *const *tri,
               const int32_t *nt, uint32_t flags, gp_mesh **out, int *status);

// device bytes gpolylla_build_halfedges takes from the pool
size_t build_footprint(int64_t nv, int64_t nt, bool inputs_on_device);
// device bytes gpolylla_mesh_batch takes from the pool for meshes of these sizes
size_t batch_footprint(const gp::LaunchCfg &cfg, const int32_t *nts, int n);

}  // namespace gprt

struct gp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    gprt::DevPool pool;
    gp::LaunchCfg cfg;
    bool profile = false;
    bool debug = false;   // runs keep snapshots of their intermediate stages
    struct Pending {
        int kernel;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare_events;
    std::vector<hipEvent_t> done_events;   // completion events of finished runs, for reuse
    hipEvent_t open_ev[gp::K_COUNT] = {};
    double kms[gp::K_COUNT] = {};
    int64_t kcount[gp::K_COUNT] = {};
    // pinned host memory: cached blocks, descriptor staging ring, and runs
    // whose results were freed before their work finished
    std::multimap<size_t, void *> pinned_free;
    struct Slot {
        void *ptr = nullptr;
        size_t bytes = 0;
        hipEvent_t ev = nullptr;
        bool armed = false;
    };
    Slot ring[4];
    int ring_next = 0;
    std::vector<gprt::RunState *> retired;
    gprt::GraphCache *graphs = nullptr;
};

struct gp_mesh {
    gp_ctx *ctx = nullptr;
    int32_t nv = 0, nt = 0;
    int64_t nflipped = 0;
    int2 *xy = nullptr;
    int32_t *org = nullptr;    // null in a compact mesh
    int32_t *twin = nullptr;   // null in a compact mesh
    // compact meshes (GP_COMPACT): see gp::MeshDesc
    int2 *org8 = nullptr;
    int16_t *twin16 = nullptr;
    int32_t *esc = nullptr;
    int32_t esc_mask = 0;
    int32_t nesc = 0;
    // renumbered meshes (GP_RENUMBER): new -> old vertex and triangle index
    int32_t *vperm = nullptr;
    int32_t *tperm = nullptr;
    size_t bytes = 0;          // device bytes the mesh holds
};

// The mesh's fields of a descriptor.
inline void mesh_desc_fill(const gp_mesh *m, gp::MeshDesc &d) {
    d.xy = m->xy;
    d.org = m->org;
    d.twin = m->twin;
    d.org8 = m->org8;
    d.twin16 = m->twin16;
    d.esc = m->esc;
    d.esc_mask = m->esc_mask;
}

namespace gprt {
// Snapshots of a debug run's intermediate stages (device memory): per mesh
// the label bytes and next'/prev' as k_relink left them (before the repair),
// and the label bytes at the end; for the run, the barrier-tip list.
struct DebugSnap {
    void *block = nullptr;
    std::vector<uint8_t *> tflag_relink, tflag_final;
    std::vector<int32_t *> next_relink, prev_relink;
    gp::ListEntry *tips = nullptr;    // cap_tips entries
    int32_t *ntips = nullptr;         // the run's tip count
    int32_t cap_tips = 0;
};

struct RunState {
    gp_ctx *ctx = nullptr;
    void *out_block = nullptr;        // outputs of every mesh of the run
    DebugSnap *dbg = nullptr;         // debug runs only
    gp::MeshCounters *host_ctrs = nullptr;  // pinned
    size_t host_ctrs_bytes = 0;
    int nmesh = 0;
    hipEvent_t done = nullptr;
    bool synced = false;
    int status = GP_OK;
    int refs = 0;
};
}  // namespace gprt

// A result is either device-resident (run != nullptr: outputs in the run's
// pool block) or host-resident (host == true: outputs in host memory that
// on_free gives back; made by the serving loop).
struct gp_result {
    gprt::RunState *run = nullptr;
    int index = 0;
    int32_t nt = 0, nv = 0;
    int64_t nflipped = 0;
    int32_t *next_o = nullptr, *prev_o = nullptr, *seeds = nullptr, *loop_off = nullptr,
            *loop_he = nullptr;
    bool host = false;
    gp_result_info hinfo{};
    std::function<void()> on_free;
};
