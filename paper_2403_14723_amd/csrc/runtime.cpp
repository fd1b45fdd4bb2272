// Host runtime behind the C ABI of include/gpolylla.h: device pool,
// per-run arenas, descriptor tables, kernel timing, build and mesh calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/gpolylla.h"
#include "gp_internal.h"

namespace {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t n, size_t a = kAlign) { return (n + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// caching device allocator: blocks are kept after release and handed out
// again for requests of up to 12.5% smaller size.  All users of one pool run
// on one stream, so reuse after release is ordered by the stream.
// ---------------------------------------------------------------------------
class DevPool {
  public:
    size_t cap = 0;
    size_t held = 0;
    size_t in_use = 0;

    int alloc(size_t n, void **p) {
        n = align_up(n ? n : kAlign);
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
        if (!p) return;
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
        held = in_use = 0;
    }

  private:
    std::multimap<size_t, void *> free_;
    std::unordered_map<void *, size_t> used_;
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

}  // namespace

// ---------------------------------------------------------------------------
// objects
// ---------------------------------------------------------------------------

struct RunState;

struct gp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    DevPool pool;
    gp::LaunchCfg cfg;
    bool profile = false;
    struct Pending {
        int kernel;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare_events;
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
    std::vector<RunState *> retired;
};

struct gp_mesh {
    gp_ctx *ctx = nullptr;
    int32_t nv = 0, nt = 0;
    int64_t nflipped = 0;
    int2 *xy = nullptr;
    int32_t *org = nullptr;
    int32_t *twin = nullptr;
};

struct RunState {
    gp_ctx *ctx = nullptr;
    void *out_block = nullptr;        // outputs of every mesh of the run
    gp::MeshCounters *host_ctrs = nullptr;  // pinned
    size_t host_ctrs_bytes = 0;
    int nmesh = 0;
    hipEvent_t done = nullptr;
    bool synced = false;
    int status = GP_OK;
    int refs = 0;
};

struct gp_result {
    RunState *run = nullptr;
    int index = 0;
    int32_t nt = 0, nv = 0;
    int64_t nflipped = 0;
    int32_t *next_o = nullptr, *prev_o = nullptr, *seeds = nullptr, *loop_off = nullptr,
            *loop_he = nullptr;
};

namespace {

#define HIP_OK(expr)                                        \
    do {                                                    \
        if ((expr) != hipSuccess) {                         \
            (void)hipGetLastError();                        \
            return GP_EHIP;                                 \
        }                                                   \
    } while (0)

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

hipEvent_t take_event(gp_ctx *c) {
    if (!c->spare_events.empty()) {
        hipEvent_t e = c->spare_events.back();
        c->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void profile_hook(void *user, int kernel, int after) {
    gp_ctx *c = static_cast<gp_ctx *>(user);
    if (!after) {
        c->open_ev[kernel] = take_event(c);
        if (c->open_ev[kernel]) (void)hipEventRecord(c->open_ev[kernel], c->stream);
    } else {
        hipEvent_t b = take_event(c);
        if (b && c->open_ev[kernel]) {
            (void)hipEventRecord(b, c->stream);
            c->pending.push_back({kernel, c->open_ev[kernel], b});
        }
        c->open_ev[kernel] = nullptr;
    }
}

// Folds finished event pairs into the per-kernel totals; pairs whose work is
// still queued stay pending.
void resolve_profile(gp_ctx *c) {
    size_t k = 0;
    for (size_t i = 0; i < c->pending.size(); i++) {
        auto &p = c->pending[i];
        hipError_t q = hipEventQuery(p.b);
        if (q == hipErrorNotReady) {
            c->pending[k++] = p;
            continue;
        }
        float ms = 0.f;
        if (q == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->kms[p.kernel] += ms;
            c->kcount[p.kernel] += 1;
        } else {
            (void)hipGetLastError();
        }
        c->spare_events.push_back(p.a);
        c->spare_events.push_back(p.b);
    }
    c->pending.resize(k);
}

void *pinned_take(gp_ctx *c, size_t n) {
    n = align_up(n ? n : kAlign);
    auto it = c->pinned_free.lower_bound(n);
    if (it != c->pinned_free.end() && it->first <= 2 * n) {
        void *p = it->second;
        c->pinned_free.erase(it);
        return p;
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void pinned_give(gp_ctx *c, void *p, size_t n) {
    if (p) c->pinned_free.emplace(align_up(n ? n : kAlign), p);
}

// Copies host bytes to device memory through a pinned staging slot.  A slot
// is reused only after the copy that last read it has completed.
hipError_t stage_to_device(gp_ctx *c, void *dst, const void *src, size_t n) {
    gp_ctx::Slot &sl = c->ring[c->ring_next];
    c->ring_next = (c->ring_next + 1) % 4;
    if (sl.armed) {
        hipError_t e = hipEventSynchronize(sl.ev);
        if (e != hipSuccess) return e;
        sl.armed = false;
    }
    if (sl.bytes < n) {
        if (sl.ptr) (void)hipHostFree(sl.ptr);
        sl.ptr = nullptr;
        sl.bytes = 0;
        size_t want = align_up(std::max<size_t>(n, 4096));
        hipError_t e = hipHostMalloc(&sl.ptr, want, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        sl.bytes = want;
    }
    if (!sl.ev) {
        hipError_t e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    std::memcpy(sl.ptr, src, n);
    hipError_t e = hipMemcpyAsync(dst, sl.ptr, n, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return e;
    e = hipEventRecord(sl.ev, c->stream);
    if (e == hipSuccess) sl.armed = true;
    return e;
}

void run_destroy(RunState *r) {
    pinned_give(r->ctx, r->host_ctrs, r->host_ctrs_bytes);
    if (r->done) (void)hipEventDestroy(r->done);
    delete r;
}

// Frees the host side of runs whose device work has finished.
void reap_retired(gp_ctx *c, bool wait) {
    auto &v = c->retired;
    size_t k = 0;
    for (size_t i = 0; i < v.size(); i++) {
        RunState *r = v[i];
        hipError_t q = wait ? hipEventSynchronize(r->done) : hipEventQuery(r->done);
        if (q == hipSuccess) {
            run_destroy(r);
        } else {
            if (q != hipErrorNotReady) (void)hipGetLastError();
            v[k++] = r;
        }
    }
    v.resize(k);
}

int run_sync(RunState *r) {
    if (r->synced) return r->status;
    DeviceGuard g(r->ctx->device);
    if (hipEventSynchronize(r->done) != hipSuccess) {
        (void)hipGetLastError();
        r->status = GP_EHIP;
    } else {
        for (int i = 0; i < r->nmesh; i++)
            if (r->host_ctrs[i].err) r->status = GP_ECORRUPT;
    }
    if (r->ctx->profile) resolve_profile(r->ctx);
    r->synced = true;
    return r->status;
}

// The last result of a run is gone: its device outputs go back to the pool
// at once (later work on the stream is ordered after this run); the host
// side waits on the retire list until the run's event has completed.
void run_unref(RunState *r) {
    if (!r || --r->refs > 0) return;
    gp_ctx *c = r->ctx;
    DeviceGuard g(c->device);
    c->pool.release(r->out_block);
    r->out_block = nullptr;
    if (r->synced || hipEventQuery(r->done) == hipSuccess) {
        run_destroy(r);
    } else {
        (void)hipGetLastError();
        c->retired.push_back(r);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *gpolylla_strerror(int code) {
    switch (code) {
        case GP_OK: return "ok";
        case GP_EINVAL: return "invalid argument (null pointer, negative count or vertex index out of range)";
        case GP_ERANGE: return "value out of range (coordinate outside [0, 2^30] or 3*nt >= 2^31)";
        case GP_EDEGEN: return "zero-area triangle";
        case GP_ENONMANIFOLD: return "non-manifold edge (more than two triangles, or a repeated directed edge)";
        case GP_ENOMEM: return "out of memory (device, pinned host, or pool cap)";
        case GP_EHIP: return "HIP runtime error";
        case GP_EAGAIN: return "queue full, try again";
        case GP_ETOOBIG: return "request larger than the server pool";
        case GP_ETIMEDOUT: return "timed out";
        case GP_ECORRUPT: return "corrupt half-edge structure (a rotation, walk or scan guard tripped)";
        default: return "unknown error";
    }
}

int gpolylla_ctx_create(int device, const gp_ctx_opts *opts, gp_ctx **out) {
    if (!out) return GP_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) {
        (void)hipGetLastError();
        return GP_EHIP;
    }
    if (device < 0 || device >= ndev) return GP_EINVAL;
    gp_ctx *c = new (std::nothrow) gp_ctx();
    if (!c) return GP_ENOMEM;
    c->device = device;
    DeviceGuard g(device);
    if (opts) {
        c->pool.cap = opts->pool_bytes;
        c->profile = opts->profile != 0;
        if (opts->block > 0) {
            if (opts->block % 64 || opts->block > 1024) {
                delete c;
                return GP_EINVAL;
            }
            c->cfg.block_label = c->cfg.block_relink = c->cfg.block_compact = opts->block;
        }
        if (opts->items > 0) {
            if (opts->items != 1 && opts->items != 2 && opts->items != 4 && opts->items != 8) {
                delete c;
                return GP_EINVAL;
            }
            c->cfg.items_label = c->cfg.items_relink = c->cfg.items_compact = opts->items;
        }
    }
    if (opts && opts->stream) {
        c->stream = static_cast<hipStream_t>(opts->stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            delete c;
            return GP_EHIP;
        }
        c->own_stream = true;
    }
    *out = c;
    return GP_OK;
}

void gpolylla_ctx_destroy(gp_ctx *c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    resolve_profile(c);
    reap_retired(c, true);
    for (auto e : c->spare_events) (void)hipEventDestroy(e);
    c->pool.destroy();
    for (auto &kv : c->pinned_free) (void)hipHostFree(kv.second);
    for (auto &sl : c->ring) {
        if (sl.ptr) (void)hipHostFree(sl.ptr);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
    }
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int gpolylla_ctx_pool_bytes(const gp_ctx *c, size_t *held, size_t *in_use) {
    if (!c) return GP_EINVAL;
    if (held) *held = c->pool.held;
    if (in_use) *in_use = c->pool.in_use;
    return GP_OK;
}

int gpolylla_ctx_sync(gp_ctx *c) {
    if (!c) return GP_EINVAL;
    DeviceGuard g(c->device);
    HIP_OK(hipStreamSynchronize(c->stream));
    if (c->profile) resolve_profile(c);
    reap_retired(c, false);
    return GP_OK;
}

int gpolylla_ctx_kernel_ms(gp_ctx *c, const char **names, double *avg_ms, int64_t *launches, int cap) {
    if (!c) return GP_EINVAL;
    int n = 0;
    for (int k = 0; k < gp::K_COUNT && n < cap; k++, n++) {
        if (names) names[n] = gp::kKernelNames[k];
        if (avg_ms) avg_ms[n] = c->kcount[k] ? c->kms[k] / (double)c->kcount[k] : 0.0;
        if (launches) launches[n] = c->kcount[k];
    }
    return n;
}

void gpolylla_ctx_kernel_reset(gp_ctx *c) {
    if (!c) return;
    for (int k = 0; k < gp::K_COUNT; k++) {
        c->kms[k] = 0;
        c->kcount[k] = 0;
    }
}

// ---------------------------------------------------------------------------
// build
// ---------------------------------------------------------------------------

int gpolylla_build_halfedges(gp_ctx *c, const int32_t *xy, int32_t nv, const int32_t *tri, int32_t nt,
                             uint32_t flags, gp_mesh **out) {
    if (!c || !out) return GP_EINVAL;
    *out = nullptr;
    if (nv < 0 || nt < 0) return GP_EINVAL;
    if ((nv > 0 && !xy) || (nt > 0 && !tri)) return GP_EINVAL;
    if (3ll * nt >= (1ll << 31)) return GP_ERANGE;
    DeviceGuard g(c->device);
    const bool in_dev = (flags & GP_IN_DEVICE) != 0;
    const int64_t nh = 3ll * nt;

    gp_mesh *m = new (std::nothrow) gp_mesh();
    if (!m) return GP_ENOMEM;
    m->ctx = c;
    m->nv = nv;
    m->nt = nt;
    int rc = GP_OK;
    void *p_xy = nullptr, *p_org = nullptr, *p_twin = nullptr, *p_tmp = nullptr;
    rc = c->pool.alloc(sizeof(int2) * (size_t)std::max<int64_t>(nv, 1), &p_xy);
    if (rc == GP_OK) rc = c->pool.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nh, 1), &p_org);
    if (rc == GP_OK) rc = c->pool.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nh, 1), &p_twin);
    const int32_t scan_tiles = gp::build_scan_tiles(nv);
    const size_t tmp_bytes = arena_bytes<int32_t>(nv + 1) * 2 + arena_bytes<int32_t>(nv + 1) +
                             arena_bytes<int32_t>(nh + 1) + arena_bytes<uint64_t>(scan_tiles) +
                             arena_bytes<int32_t>(4) + arena_bytes<unsigned long long>(1) +
                             (in_dev ? 0 : arena_bytes<int32_t>(nh + 1));
    if (rc == GP_OK) rc = c->pool.alloc(tmp_bytes, &p_tmp);
    if (rc != GP_OK) {
        c->pool.release(p_xy);
        c->pool.release(p_org);
        c->pool.release(p_twin);
        c->pool.release(p_tmp);
        delete m;
        return rc;
    }
    m->xy = static_cast<int2 *>(p_xy);
    m->org = static_cast<int32_t *>(p_org);
    m->twin = static_cast<int32_t *>(p_twin);
    Arena a{static_cast<char *>(p_tmp), tmp_bytes, 0};
    gp::BuildBuffers b{};
    b.nv = nv;
    b.nt = nt;
    b.org = m->org;
    b.twin = m->twin;
    b.deg = a.take<int32_t>(nv + 1);
    b.fill = a.take<int32_t>(nv + 1);
    b.vstart = a.take<int32_t>(nv + 1);
    b.bucket = a.take<int32_t>(nh + 1);
    b.scan_status = a.take<uint64_t>(scan_tiles);
    int32_t *small = a.take<int32_t>(4);
    b.scan_ctr = small;
    b.nflipped = small + 1;
    b.err_key = a.take<unsigned long long>(1);
    int32_t *tri_dev = in_dev ? const_cast<int32_t *>(tri) : a.take<int32_t>(nh + 1);
    b.xy = m->xy;
    b.tri = tri_dev;

    auto fail = [&](int code) {
        (void)hipStreamSynchronize(c->stream);
        c->pool.release(p_tmp);
        gpolylla_mesh_free(m);
        return code;
    };
    hipStream_t s = c->stream;
    const hipMemcpyKind kind = in_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (nv > 0 && hipMemcpyAsync(m->xy, xy, sizeof(int2) * (size_t)nv, kind, s) != hipSuccess)
        return (void)hipGetLastError(), fail(GP_EHIP);
    if (!in_dev && nt > 0 &&
        hipMemcpyAsync(tri_dev, tri, sizeof(int32_t) * (size_t)nh, hipMemcpyHostToDevice, s) != hipSuccess)
        return (void)hipGetLastError(), fail(GP_EHIP);
    if (hipMemsetAsync(b.deg, 0, sizeof(int32_t) * (size_t)(nv + 1), s) != hipSuccess ||
        hipMemsetAsync(b.fill, 0, sizeof(int32_t) * (size_t)(nv + 1), s) != hipSuccess ||
        hipMemsetAsync(b.scan_status, 0, sizeof(uint64_t) * (size_t)scan_tiles, s) != hipSuccess ||
        hipMemsetAsync(small, 0, sizeof(int32_t) * 4, s) != hipSuccess ||
        hipMemsetAsync(b.err_key, 0xff, sizeof(unsigned long long), s) != hipSuccess)
        return (void)hipGetLastError(), fail(GP_EHIP);
    if (gp::launch_build_orient(b, s) != hipSuccess) return (void)hipGetLastError(), fail(GP_EHIP);
    unsigned long long key = ~0ull;
    if (hipMemcpyAsync(&key, b.err_key, sizeof(key), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return (void)hipGetLastError(), fail(GP_EHIP);
    if (key != ~0ull) return fail(-(int)(key & 0xff));
    if (gp::launch_build_link(b, s) != hipSuccess) return (void)hipGetLastError(), fail(GP_EHIP);
    int32_t nflip = 0;
    if (hipMemcpyAsync(&key, b.err_key, sizeof(key), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&nflip, b.nflipped, sizeof(nflip), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return (void)hipGetLastError(), fail(GP_EHIP);
    if (key != ~0ull) return fail(-(int)(key & 0xff));
    m->nflipped = nflip;
    c->pool.release(p_tmp);
    *out = m;
    return GP_OK;
}

int gpolylla_mesh_copy(const gp_mesh *m, int32_t *org, int32_t *twin, int64_t *nflipped) {
    if (!m) return GP_EINVAL;
    DeviceGuard g(m->ctx->device);
    size_t n = sizeof(int32_t) * 3 * (size_t)m->nt;
    if (org && n) HIP_OK(hipMemcpy(org, m->org, n, hipMemcpyDeviceToHost));
    if (twin && n) HIP_OK(hipMemcpy(twin, m->twin, n, hipMemcpyDeviceToHost));
    if (nflipped) *nflipped = m->nflipped;
    return GP_OK;
}

int gpolylla_mesh_size(const gp_mesh *m, int32_t *nv, int32_t *nt) {
    if (!m) return GP_EINVAL;
    if (nv) *nv = m->nv;
    if (nt) *nt = m->nt;
    return GP_OK;
}

void gpolylla_mesh_free(gp_mesh *m) {
    if (!m) return;
    DeviceGuard g(m->ctx->device);
    // stream-ordered: later work on the context stream may reuse the blocks
    m->ctx->pool.release(m->xy);
    m->ctx->pool.release(m->org);
    m->ctx->pool.release(m->twin);
    delete m;
}

// ---------------------------------------------------------------------------
// meshing
// ---------------------------------------------------------------------------

int gpolylla_mesh_batch(gp_ctx *c, const gp_mesh *const *meshes, int32_t n, uint32_t out_flags,
                        gp_result **out) {
    if (!c || !out || n < 0 || (n > 0 && !meshes)) return GP_EINVAL;
    for (int i = 0; i < n; i++) {
        out[i] = nullptr;
        if (!meshes[i] || meshes[i]->ctx != c) return GP_EINVAL;
    }
    if (n == 0) return GP_OK;
    DeviceGuard g(c->device);
    const gp::LaunchCfg &cfg = c->cfg;
    const int64_t tt = (int64_t)cfg.block_label * cfg.items_label;
    const int64_t th = (int64_t)cfg.block_relink * cfg.items_relink;
    const int64_t tc = (int64_t)cfg.block_compact * cfg.items_compact;

    // tile spaces and capacities
    std::vector<gp::MeshDesc> descs(n);
    int64_t tri_tiles = 0, he_tiles = 0, cmp_tiles = 0, cap_tips = 0, out_bytes = 0, tmp_mesh = 0;
    for (int i = 0; i < n; i++) {
        const gp_mesh *m = meshes[i];
        descs[i].nt = m->nt;
        descs[i].nv = m->nv;
        descs[i].tri_tile0 = (int32_t)tri_tiles;
        descs[i].he_tile0 = (int32_t)he_tiles;
        descs[i].cmp_tile0 = (int32_t)cmp_tiles;
        tri_tiles += gp::tiles_for(m->nt, tt);
        he_tiles += gp::tiles_for(3ll * m->nt, th);
        cmp_tiles += gp::tiles_for(m->nt, tc);
        cap_tips += m->nt / 2 + 2;   // tips are interior vertices: at most T/2 + 1
        const int64_t nh = 3ll * m->nt;
        out_bytes += 3 * arena_bytes<int32_t>(nh + 1) + arena_bytes<int32_t>(m->nt + 1) +
                     arena_bytes<int32_t>(m->nt + 2);
        tmp_mesh += arena_bytes<uint8_t>(align_up(m->nt + 4, 4)) + arena_bytes<uint8_t>(m->nt + 1);
    }
    if (tri_tiles > 0x7fffffff || he_tiles > 0x7fffffff || cap_tips > (1ll << 30)) return GP_ERANGE;
    const int64_t cap_cands = 2 * cap_tips, cap_fix = 2 * cap_tips;
    const size_t tmp_bytes = (size_t)tmp_mesh + arena_bytes<gp::MeshDesc>(n) + arena_bytes<gp::RunCounters>(1) +
                             arena_bytes<gp::MeshCounters>(n) + arena_bytes<gp::ListEntry>(cap_tips) +
                             arena_bytes<gp::ListEntry>(cap_cands) + arena_bytes<gp::ListEntry>(cap_fix) +
                             arena_bytes<uint64_t>(cmp_tiles);

    RunState *r = new (std::nothrow) RunState();
    if (!r) return GP_ENOMEM;
    r->ctx = c;
    r->nmesh = n;
    void *p_tmp = nullptr;
    int rc = c->pool.alloc((size_t)out_bytes, &r->out_block);
    if (rc == GP_OK) rc = c->pool.alloc(tmp_bytes, &p_tmp);
    reap_retired(c, false);
    if (rc == GP_OK) {
        r->host_ctrs_bytes = sizeof(gp::MeshCounters) * n;
        r->host_ctrs = static_cast<gp::MeshCounters *>(pinned_take(c, r->host_ctrs_bytes));
        if (!r->host_ctrs) rc = GP_ENOMEM;
    }
    if (rc == GP_OK && hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        r->done = nullptr;
        rc = GP_EHIP;
    }
    if (rc != GP_OK) {
        c->pool.release(r->out_block);
        c->pool.release(p_tmp);
        run_destroy(r);
        return rc;
    }
    Arena ao{static_cast<char *>(r->out_block), (size_t)out_bytes, 0};
    Arena at{static_cast<char *>(p_tmp), tmp_bytes, 0};
    std::vector<gp_result *> res(n, nullptr);
    gp::MeshDesc *d_descs = at.take<gp::MeshDesc>(n);
    gp::RunBuffers rb{};
    rb.descs = d_descs;
    rb.nmesh = n;
    rb.tri_tiles = (int32_t)tri_tiles;
    rb.he_tiles = (int32_t)he_tiles;
    rb.cmp_tiles = (int32_t)cmp_tiles;
    rb.rc = at.take<gp::RunCounters>(1);
    rb.ctrs = at.take<gp::MeshCounters>(n);
    rb.tips = at.take<gp::ListEntry>(cap_tips);
    rb.cands = at.take<gp::ListEntry>(cap_cands);
    rb.fixes = at.take<gp::ListEntry>(cap_fix);
    rb.cap_tips = (int32_t)cap_tips;
    rb.cap_cands = (int32_t)cap_cands;
    rb.cap_fix = (int32_t)cap_fix;
    rb.status = at.take<uint64_t>(cmp_tiles);
    for (int i = 0; i < n; i++) {
        const gp_mesh *m = meshes[i];
        const int64_t nh = 3ll * m->nt;
        gp_result *x = new (std::nothrow) gp_result();
        if (!x) {
            for (auto q : res) delete q;
            c->pool.release(r->out_block);
            c->pool.release(p_tmp);
            run_destroy(r);
            return GP_ENOMEM;
        }
        x->run = r;
        x->index = i;
        x->nt = m->nt;
        x->nv = m->nv;
        x->nflipped = m->nflipped;
        x->next_o = ao.take<int32_t>(nh + 1);
        x->prev_o = ao.take<int32_t>(nh + 1);
        x->loop_he = ao.take<int32_t>(nh + 1);
        x->seeds = ao.take<int32_t>(m->nt + 1);
        x->loop_off = ao.take<int32_t>(m->nt + 2);
        res[i] = x;
        gp::MeshDesc &d = descs[i];
        d.xy = m->xy;
        d.org = m->org;
        d.twin = m->twin;
        d.next_o = x->next_o;
        d.prev_o = x->prev_o;
        d.seeds = x->seeds;
        d.loop_off = x->loop_off;
        d.loop_he = x->loop_he;
        d.tflag = at.take<uint8_t>(align_up(m->nt + 4, 4));
        d.pl = at.take<uint8_t>(m->nt + 1);
        d.ctr = rb.ctrs + i;
    }
    // descriptor table: pinned staging, stream-ordered copy
    hipStream_t s = c->stream;
    int err = GP_OK;
    if (stage_to_device(c, d_descs, descs.data(), sizeof(gp::MeshDesc) * n) != hipSuccess) err = GP_EHIP;
    if (err == GP_OK &&
        gp::launch_pipeline(cfg, rb, s, c->profile ? profile_hook : nullptr, c) != hipSuccess)
        err = GP_EHIP;
    if (err == GP_OK && (hipMemcpyAsync(r->host_ctrs, rb.ctrs, sizeof(gp::MeshCounters) * n,
                                        hipMemcpyDeviceToHost, s) != hipSuccess ||
                         hipEventRecord(r->done, s) != hipSuccess))
        err = GP_EHIP;
    // temporaries go back to the pool; later users are ordered after this run
    c->pool.release(p_tmp);
    if (err != GP_OK) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        for (auto q : res) delete q;
        c->pool.release(r->out_block);
        run_destroy(r);
        return err;
    }
    r->refs = n;
    if (!(out_flags & GP_ASYNC)) {
        int st = run_sync(r);
        if (st != GP_OK) {
            for (auto q : res) {
                q->run = nullptr;
                delete q;
            }
            r->refs = 1;
            run_unref(r);
            return st;
        }
    }
    for (int i = 0; i < n; i++) out[i] = res[i];
    return GP_OK;
}

int gpolylla_mesh(gp_ctx *c, const gp_mesh *m, uint32_t out_flags, gp_result **out) {
    if (!m) return GP_EINVAL;
    return gpolylla_mesh_batch(c, &m, 1, out_flags, out);
}

int gpolylla_result_info(gp_result *x, gp_result_info *info) {
    if (!x || !info || !x->run) return GP_EINVAL;
    int st = run_sync(x->run);
    if (st != GP_OK) return st;
    const gp::MeshCounters &k = x->run->host_ctrs[x->index];
    info->nt = x->nt;
    info->nv = x->nv;
    info->nh = 3ll * x->nt;
    info->npoly = k.npoly;
    info->nloop_he = k.nloop;
    info->ntips = k.ntips;
    info->nmiddle = k.nmiddle;
    // every terminal edge gives one region, every distinct middle edge splits
    // one region in two
    info->nterminal = (int64_t)k.npoly - k.nmiddle;
    info->nties = k.nties;
    info->nflipped = x->nflipped;
    return GP_OK;
}

int gpolylla_result_copy(gp_result *x, int32_t *next, int32_t *prev, int32_t *seeds, int32_t *loop_off,
                         int32_t *loop_he) {
    gp_result_info info;
    int st = gpolylla_result_info(x, &info);
    if (st != GP_OK) return st;
    DeviceGuard g(x->run->ctx->device);
    hipStream_t s = x->run->ctx->stream;
    const size_t nh = (size_t)info.nh;
    if (next && nh) HIP_OK(hipMemcpyAsync(next, x->next_o, 4 * nh, hipMemcpyDeviceToHost, s));
    if (prev && nh) HIP_OK(hipMemcpyAsync(prev, x->prev_o, 4 * nh, hipMemcpyDeviceToHost, s));
    if (seeds && info.npoly) HIP_OK(hipMemcpyAsync(seeds, x->seeds, 4 * (size_t)info.npoly, hipMemcpyDeviceToHost, s));
    if (loop_off)
        HIP_OK(hipMemcpyAsync(loop_off, x->loop_off, 4 * (size_t)(info.npoly + 1), hipMemcpyDeviceToHost, s));
    if (loop_he && info.nloop_he)
        HIP_OK(hipMemcpyAsync(loop_he, x->loop_he, 4 * (size_t)info.nloop_he, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return GP_OK;
}

int gpolylla_result_device(gp_result *x, gp_result_dev *dev) {
    if (!x || !dev || !x->run) return GP_EINVAL;
    dev->next = x->next_o;
    dev->prev = x->prev_o;
    dev->seeds = x->seeds;
    dev->loop_off = x->loop_off;
    dev->loop_he = x->loop_he;
    return GP_OK;
}

void gpolylla_result_free(gp_result *x) {
    if (!x) return;
    run_unref(x->run);
    delete x;
}

}  // extern "C"
