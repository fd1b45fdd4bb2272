// Host runtime behind the C ABI of include/gpolylla.h: device pool,
// per-run arenas, descriptor tables, kernel timing, build and mesh calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "runtime_internal.h"

using namespace gprt;

namespace gprt {

void *pinned_take(gp_ctx *c, size_t n) {
    n = align_up(n ? n : kAlign);
    auto it = c->pinned_free.lower_bound(n);
    if (it != c->pinned_free.end() && it->first <= 2 * n) {
        void *p = it->second;
        c->pinned_free.erase(it);
        return p;
    }
    void *p = nullptr;
    // coherent: the device writes the run counters here with a kernel
    if (hipHostMalloc(&p, n, hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void pinned_give(gp_ctx *c, void *p, size_t n) {
    if (p) c->pinned_free.emplace(align_up(n ? n : kAlign), p);
}

}  // namespace gprt

namespace {

#define HIP_OK(expr)                                        \
    do {                                                    \
        if ((expr) != hipSuccess) {                         \
            (void)hipGetLastError();                        \
            return GP_EHIP;                                 \
        }                                                   \
    } while (0)

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

// The launch hook of a debug run: after k_relink the label bytes, next',
// prev' and the tip list are copied aside (in stream order, so before the
// repair changes them); after the last kernel the label bytes again.
struct DebugHook {
    gp_ctx *c;
    DebugSnap *d;
    const gp::RunBuffers *rb;
    std::vector<gp_result *> *res;
    const std::vector<uint8_t *> *tflag;
};

void debug_hook(void *user, int kernel, int after) {
    DebugHook *h = static_cast<DebugHook *>(user);
    if (h->c->profile) profile_hook(h->c, kernel, after);
    if (!after) return;
    hipStream_t s = h->c->stream;
    const int n = (int)h->res->size();
    if (kernel == gp::K_RELINK) {
        for (int i = 0; i < n; i++) {
            const gp_result *x = (*h->res)[i];
            const size_t nt = (size_t)x->nt, nh = 3 * nt;
            if (nt) (void)hipMemcpyAsync(h->d->tflag_relink[i], (*h->tflag)[i], nt, hipMemcpyDeviceToDevice, s);
            if (nh) {
                (void)hipMemcpyAsync(h->d->next_relink[i], x->next_o, 4 * nh, hipMemcpyDeviceToDevice, s);
                (void)hipMemcpyAsync(h->d->prev_relink[i], x->prev_o, 4 * nh, hipMemcpyDeviceToDevice, s);
            }
        }
        (void)hipMemcpyAsync(h->d->tips, h->rb->tips, sizeof(gp::ListEntry) * (size_t)h->d->cap_tips,
                             hipMemcpyDeviceToDevice, s);
        (void)hipMemcpyAsync(h->d->ntips, &h->rb->rc->ntips, sizeof(int32_t), hipMemcpyDeviceToDevice, s);
    } else if (kernel == gp::K_EMIT) {
        for (int i = 0; i < n; i++) {
            const size_t nt = (size_t)(*h->res)[i]->nt;
            if (nt) (void)hipMemcpyAsync(h->d->tflag_final[i], (*h->tflag)[i], nt, hipMemcpyDeviceToDevice, s);
        }
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

// Copies host bytes to device memory through a pinned staging slot, read by a
// small copy kernel in stream order (the runtime's asynchronous copy of such
// small tables stalled the host for milliseconds now and then, leaving the
// device idle).  A slot is reused only after the copy that last read it has
// completed; slots are coherent, so the kernel never sees a cached copy.
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
        hipError_t e = hipHostMalloc(&sl.ptr, want, hipHostMallocCoherent);
        if (e != hipSuccess) return e;
        sl.bytes = want;
    }
    if (!sl.ev) {
        hipError_t e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    std::memcpy(sl.ptr, src, n);
    hipError_t e = gp::launch_copy_words(dst, sl.ptr, align_up(n, 4), c->stream);
    if (e != hipSuccess) return e;
    e = hipEventRecord(sl.ev, c->stream);
    if (e == hipSuccess) sl.armed = true;
    return e;
}

void run_destroy(RunState *r) {
    pinned_give(r->ctx, r->host_ctrs, r->host_ctrs_bytes);
    delete r->dbg;
    if (r->done) r->ctx->done_events.push_back(r->done);   // completed (or never recorded): reusable
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
    if (r->dbg) {
        c->pool.release(r->dbg->block);
        r->dbg->block = nullptr;
    }
    if (r->synced || hipEventQuery(r->done) == hipSuccess) {
        run_destroy(r);
    } else {
        (void)hipGetLastError();
        c->retired.push_back(r);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// run planning: tile spaces, list capacities, scratch layout
// ---------------------------------------------------------------------------

namespace {

// Sizes of one run over meshes of nts[0..n) triangles.  No allocation: the
// no-allocation entry point plans its single mesh with this directly.
struct PlanSizes {
    int64_t tri_tiles = 0, he_tiles = 0, cmp_tiles = 0, cap_tips = 0, cap_fix = 0;
    int64_t walk_cap = 0, emit_cap = 0, wbuf_cap = 0;
    size_t out_bytes = 0, tmp_bytes = 0, tmp_mesh = 0;
};

// Fills the sizes and tile offsets of descs[0..n) (nt, nv, *_tile0) and *p.
int plan_core(const gp::LaunchCfg &cfg, const int32_t *nts, const int32_t *nvs, int n, gp::MeshDesc *descs,
              PlanSizes *p) {
    const int64_t tt = (int64_t)cfg.block_label * cfg.items_label;
    const int64_t th = (int64_t)cfg.block_relink * cfg.items_relink;
    const int64_t tc = (int64_t)cfg.block_compact * cfg.items_compact;
    *p = PlanSizes{};
    int64_t total_nt = 0;
    for (int i = 0; i < n; i++) {
        const int32_t nt = nts[i];
        gp::MeshDesc &d = descs[i];
        d = gp::MeshDesc{};
        d.nt = nt;
        d.nv = nvs ? nvs[i] : 0;
        d.tri_tile0 = (int32_t)p->tri_tiles;
        d.he_tile0 = (int32_t)p->he_tiles;
        d.cmp_tile0 = (int32_t)p->cmp_tiles;
        p->tri_tiles += gp::tiles_for(nt, tt);
        p->he_tiles += gp::tiles_for(nt, th);
        p->cmp_tiles += gp::tiles_for(nt, tc);
        p->cap_tips += nt / 2 + 2;   // tips are interior vertices: at most T/2 + 1
        const int64_t nh = 3ll * nt;
        p->out_bytes += 3 * arena_bytes<int32_t>(nh + 1) + arena_bytes<int32_t>(nt + 1) +
                        arena_bytes<int32_t>(nt + 2);
        p->tmp_mesh += 2 * arena_bytes<uint8_t>(align_up(nt + 4, 4)) + arena_bytes<int32_t>(nt + 1);
        total_nt += nt;
        if (p->tri_tiles > 0x7fffffff || p->he_tiles > 0x7fffffff || p->cap_tips > (1ll << 30)) return GP_ERANGE;
    }
    p->cap_fix = 2 * p->cap_tips;
    // striped lists, sized for the worst case: every triangle of a tile holds
    // a seed (walk) or a loop minimum (emit); repair seeds spread evenly
    const int64_t S = gp::kStripes;
    p->walk_cap = (p->he_tiles + S - 1) / S * th + (2 * p->cap_tips + S - 1) / S + 2;
    p->emit_cap = (p->cmp_tiles + S - 1) / S * tc;
    // walked loops: at most 3T half-edges in all (each loop is stored once)
    // plus one rotation index per loop; slack for uneven stripes
    p->wbuf_cap = align_up((4 * total_nt + S - 1) / S + 4096, 4);
    if (p->walk_cap * S > 0x7fffffff || p->emit_cap * S > 0x7fffffff || p->wbuf_cap * S > 0x7fffffff)
        return GP_ERANGE;
    p->tmp_bytes = p->tmp_mesh + arena_bytes<gp::MeshDesc>(n) + arena_bytes<gp::RunCounters>(1) +
                   arena_bytes<gp::MeshCounters>(n) + arena_bytes<gp::ListEntry>(p->cap_tips) +
                   arena_bytes<gp::ListEntry>(p->cap_fix) + 2 * arena_bytes<uint64_t>(p->cmp_tiles) +
                   arena_bytes<gp::ListEntry>(p->walk_cap * S) + arena_bytes<gp::EmitEntry>(p->emit_cap * S) +
                   arena_bytes<int32_t>(p->wbuf_cap * S + 32) + 3 * arena_bytes<int32_t>(S * gp::kStripePad);
    return GP_OK;
}

struct Plan : PlanSizes {
    std::vector<gp::MeshDesc> descs;   // sizes and tile offsets filled in
    std::vector<int32_t> nts;
    bool compact = false;              // some mesh is in the compact encoding
};

int make_plan(const gp::LaunchCfg &cfg, const gp_mesh *const *meshes, int n, Plan *p) {
    p->descs.assign(n, gp::MeshDesc{});
    p->nts.resize(n);
    p->compact = false;
    std::vector<int32_t> nvs(n);
    for (int i = 0; i < n; i++) {
        p->nts[i] = meshes[i]->nt;
        nvs[i] = meshes[i]->nv;
        p->compact |= meshes[i]->org8 != nullptr;
    }
    return plan_core(cfg, p->nts.data(), nvs.data(), n, p->descs.data(), p);
}

// Carves the run scratch out of `block` (PlanSizes::tmp_bytes bytes): the
// run's buffers into *rb, each mesh's label, loop and walk-position arrays
// into tflag[i], pl[i], lpos[i].  descs holds the planned tile offsets.
void layout_scratch(const PlanSizes &p, const gp::MeshDesc *descs, int n, void *block, gp::RunBuffers *rb,
                    uint8_t **tflag, uint8_t **pl, int32_t **lpos) {
    const int64_t S = gp::kStripes;
    Arena at{static_cast<char *>(block), p.tmp_bytes, 0};
    *rb = gp::RunBuffers{};
    rb->descs = at.take<gp::MeshDesc>(n);
    rb->nmesh = n;
    rb->tri_tiles = (int32_t)p.tri_tiles;
    rb->he_tiles = (int32_t)p.he_tiles;
    rb->cmp_tiles = (int32_t)p.cmp_tiles;
    rb->rc = at.take<gp::RunCounters>(1);
    rb->ctrs = at.take<gp::MeshCounters>(n);
    rb->tips = at.take<gp::ListEntry>(p.cap_tips);
    rb->fixes = at.take<gp::ListEntry>(p.cap_fix);
    rb->cap_tips = (int32_t)p.cap_tips;
    rb->cap_fix = (int32_t)p.cap_fix;
    rb->status = at.take<uint64_t>(p.cmp_tiles);
    rb->cpre = at.take<uint64_t>(p.cmp_tiles);
    {
        int64_t mc = 1;
        for (int i = 0; i < n; i++) {
            const int64_t end = i + 1 < n ? descs[i + 1].cmp_tile0 : p.cmp_tiles;
            const int64_t nt_tiles = end - descs[i].cmp_tile0;
            mc = std::max<int64_t>(mc, (nt_tiles + gp::kScanChunk - 1) / gp::kScanChunk);
        }
        rb->max_chunks = (int32_t)mc;
    }
    rb->walk = at.take<gp::ListEntry>(p.walk_cap * S);
    rb->walk_counts = at.take<int32_t>(S * gp::kStripePad);
    rb->walk_cap = (int32_t)p.walk_cap;
    rb->emit = at.take<gp::EmitEntry>(p.emit_cap * S);
    rb->emit_counts = at.take<int32_t>(S * gp::kStripePad);
    rb->emit_cap = (int32_t)p.emit_cap;
    rb->wbuf = at.take<int32_t>(p.wbuf_cap * S + 32);   // + a 16-byte-group overread at the end
    rb->wbuf_counts = at.take<int32_t>(S * gp::kStripePad);
    rb->wbuf_cap = (int32_t)p.wbuf_cap;
    rb->max_nt = 0;
    rb->chain_only = false;
    for (int i = 0; i < n; i++) {
        rb->max_nt = std::max(rb->max_nt, descs[i].nt);
        tflag[i] = at.take<uint8_t>(align_up(descs[i].nt + 4, 4));
        pl[i] = at.take<uint8_t>(align_up(descs[i].nt + 4, 4));   // whole words: k_walk claims by OR
        lpos[i] = at.take<int32_t>(descs[i].nt + 1);
    }
}

}  // namespace

namespace gprt {

namespace {

// One half-edge build, in three stages around the two checks of its inputs
// (orientation and indices first, then the twin matching), so that many
// builds can share each host check.
struct BuildJob {
    gp_mesh *m = nullptr;
    void *p_tmp = nullptr;
    gp::BuildBuffers b{};
    unsigned long long *key_h = nullptr;   // pinned: the error key after a stage
    int32_t *nflip_h = nullptr;            // pinned: triangles flipped to CCW
    int rc = GP_OK;
};

void build_abort(gp_ctx *c, BuildJob &j) {
    if (j.p_tmp) c->pool.release(j.p_tmp);
    j.p_tmp = nullptr;
    if (j.m) gpolylla_mesh_free(j.m);
    j.m = nullptr;
}

// Stage 0: allocation, input copies, clears and the orientation kernels
// (which also check every index and coordinate), all queued.
int build_stage0(gp_ctx *c, const int32_t *xy, int32_t nv, const int32_t *tri, int32_t nt, uint32_t flags,
                 BuildJob &j) {
    if (nv < 0 || nt < 0) return GP_EINVAL;
    if ((nv > 0 && !xy) || (nt > 0 && !tri)) return GP_EINVAL;
    if (3ll * nt >= (1ll << 31)) return GP_ERANGE;
    const bool in_dev = (flags & GP_IN_DEVICE) != 0;
    const int64_t nh = 3ll * nt;
    gp_mesh *m = new (std::nothrow) gp_mesh();
    if (!m) return GP_ENOMEM;
    m->ctx = c;
    m->nv = nv;
    m->nt = nt;
    j.m = m;
    void *p_xy = nullptr, *p_org = nullptr, *p_twin = nullptr;
    int rc = c->pool.alloc(sizeof(int2) * (size_t)std::max<int64_t>(nv, 1), &p_xy);
    m->xy = static_cast<int2 *>(p_xy);
    if (rc == GP_OK) rc = c->pool.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nh, 1), &p_org);
    m->org = static_cast<int32_t *>(p_org);
    if (rc == GP_OK) rc = c->pool.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nh, 1), &p_twin);
    m->twin = static_cast<int32_t *>(p_twin);
    const int32_t scan_tiles = gp::build_scan_tiles(nv);
    const size_t tmp_bytes = arena_bytes<int32_t>(nv + 1) * 2 + arena_bytes<int32_t>(nv + 1) +
                             arena_bytes<int2>(nh + 1) + arena_bytes<uint64_t>(scan_tiles) +
                             arena_bytes<int32_t>(4) + arena_bytes<unsigned long long>(1) +
                             (in_dev ? 0 : arena_bytes<int32_t>(nh + 1));
    if (rc == GP_OK) rc = c->pool.alloc(tmp_bytes, &j.p_tmp);
    if (rc != GP_OK) return rc;
    Arena a{static_cast<char *>(j.p_tmp), tmp_bytes, 0};
    gp::BuildBuffers &b = j.b;
    b.nv = nv;
    b.nt = nt;
    b.org = m->org;
    b.twin = m->twin;
    b.deg = a.take<int32_t>(nv + 1);
    b.fill = a.take<int32_t>(nv + 1);
    b.vstart = a.take<int32_t>(nv + 1);
    b.bucket = a.take<int2>(nh + 1);
    b.scan_status = a.take<uint64_t>(scan_tiles);
    int32_t *small = a.take<int32_t>(4);
    b.scan_ctr = small;
    b.nflipped = small + 1;
    b.err_key = a.take<unsigned long long>(1);
    int32_t *tri_dev = in_dev ? const_cast<int32_t *>(tri) : a.take<int32_t>(nh + 1);
    b.xy = m->xy;
    b.tri = tri_dev;
    hipStream_t s = c->stream;
    const hipMemcpyKind kind = in_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if ((nv > 0 && hipMemcpyAsync(m->xy, xy, sizeof(int2) * (size_t)nv, kind, s) != hipSuccess) ||
        (!in_dev && nt > 0 &&
         hipMemcpyAsync(tri_dev, tri, sizeof(int32_t) * (size_t)nh, hipMemcpyHostToDevice, s) != hipSuccess) ||
        hipMemsetAsync(b.deg, 0, sizeof(int32_t) * (size_t)(nv + 1), s) != hipSuccess ||
        hipMemsetAsync(b.fill, 0, sizeof(int32_t) * (size_t)(nv + 1), s) != hipSuccess ||
        hipMemsetAsync(b.scan_status, 0, sizeof(uint64_t) * (size_t)scan_tiles, s) != hipSuccess ||
        hipMemsetAsync(small, 0, sizeof(int32_t) * 4, s) != hipSuccess ||
        hipMemsetAsync(b.err_key, 0xff, sizeof(unsigned long long), s) != hipSuccess ||
        gp::launch_build_orient(b, s) != hipSuccess ||
        hipMemcpyAsync(j.key_h, b.err_key, sizeof(unsigned long long), hipMemcpyDeviceToHost, s) != hipSuccess) {
        (void)hipGetLastError();
        return GP_EHIP;
    }
    return GP_OK;
}

// Stage 1 (after the stream has drained stage 0): the inputs passed their
// checks; queue the twin matching and the readbacks of its checks.
int build_stage1(gp_ctx *c, BuildJob &j) {
    if (*j.key_h != ~0ull) return -(int)(*j.key_h & 0xff);
    hipStream_t s = c->stream;
    if (gp::launch_build_link(j.b, s) != hipSuccess ||
        hipMemcpyAsync(j.key_h, j.b.err_key, sizeof(unsigned long long), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(j.nflip_h, j.b.nflipped, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess) {
        (void)hipGetLastError();
        return GP_EHIP;
    }
    return GP_OK;
}

// Stage 2 (after the stream has drained stage 1): the mesh is complete.
int build_stage2(gp_ctx *c, BuildJob &j) {
    if (*j.key_h != ~0ull) return -(int)(*j.key_h & 0xff);
    j.m->nflipped = *j.nflip_h;
    j.m->bytes = align_up(sizeof(int2) * (size_t)std::max(j.m->nv, 1)) +
                 2 * align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(3ll * j.m->nt, 1));
    c->pool.release(j.p_tmp);
    j.p_tmp = nullptr;
    return GP_OK;
}

// Re-encodes a built mesh compactly (see gp::MeshDesc) and frees its int32
// corners and twins.  host: 4 bytes of pinned scratch.
int compact_mesh(gp_ctx *c, gp_mesh *m, int32_t *host) {
    const int64_t nt = m->nt, nh = 3 * nt;
    void *p8 = nullptr, *p16 = nullptr, *pe = nullptr, *pn = nullptr;
    int rc = c->pool.alloc(sizeof(int2) * (size_t)std::max<int64_t>(nt, 1), &p8);
    if (rc == GP_OK) rc = c->pool.alloc(sizeof(int16_t) * (size_t)std::max<int64_t>(nh, 1), &p16);
    if (rc == GP_OK) rc = c->pool.alloc(sizeof(int32_t), &pn);
    gp::CompactBuffers cb{};
    cb.org = m->org;
    cb.twin = m->twin;
    cb.nt = m->nt;
    cb.org8 = static_cast<int2 *>(p8);
    cb.twin16 = static_cast<int16_t *>(p16);
    cb.nesc = static_cast<int32_t *>(pn);
    hipStream_t s = c->stream;
    if (rc == GP_OK &&
        (hipMemsetAsync(cb.nesc, 0, sizeof(int32_t), s) != hipSuccess ||
         gp::launch_compact_encode(cb, s) != hipSuccess ||
         hipMemcpyAsync(host, cb.nesc, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess)) {
        (void)hipGetLastError();
        rc = GP_EHIP;
    }
    int32_t slots = 2;   // a power of two at least twice the escapes
    if (rc == GP_OK) {
        while (slots < 2 * (int64_t)*host) slots *= 2;
        rc = c->pool.alloc(2 * sizeof(int32_t) * (size_t)slots, &pe);
    }
    cb.esc = static_cast<int32_t *>(pe);
    cb.esc_mask = slots - 1;
    if (rc == GP_OK &&
        (gp::launch_compact_escapes(cb, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)) {
        (void)hipGetLastError();
        rc = GP_EHIP;
    }
    c->pool.release(pn);
    if (rc != GP_OK) {
        (void)hipStreamSynchronize(s);
        c->pool.release(p8);
        c->pool.release(p16);
        c->pool.release(pe);
        return rc;
    }
    m->nesc = *host;
    c->pool.release(m->org);
    c->pool.release(m->twin);
    m->org = m->twin = nullptr;
    m->org8 = cb.org8;
    m->twin16 = cb.twin16;
    m->esc = cb.esc;
    m->esc_mask = cb.esc_mask;
    m->bytes = align_up(sizeof(int2) * (size_t)std::max(m->nv, 1)) +
               align_up(sizeof(int2) * (size_t)std::max<int64_t>(nt, 1)) +
               align_up(sizeof(int16_t) * (size_t)std::max<int64_t>(nh, 1)) +
               align_up(2 * sizeof(int32_t) * (size_t)slots);
    return GP_OK;
}

// The renumbered copy of one build's input (GP_RENUMBER): device arrays in
// the new numbering, the two maps, and the scratch they took.
struct Renumbered {
    void *xy = nullptr, *tri = nullptr, *vperm = nullptr, *tperm = nullptr, *tmp = nullptr;
    void *in_xy = nullptr, *in_tri = nullptr;   // uploads of host inputs
};

void renumbered_free(gp_ctx *c, Renumbered &r, bool keep_maps) {
    for (void *p : {r.xy, r.tri, r.tmp, r.in_xy, r.in_tri}) c->pool.release(p);
    if (!keep_maps) {
        c->pool.release(r.vperm);
        c->pool.release(r.tperm);
    }
    r = Renumbered{};
}

// Queues the renumbering of one input on the context's stream.
int renumber_input(gp_ctx *c, const int32_t *xy, int32_t nv, const int32_t *tri, int32_t nt, bool in_dev,
                   Renumbered &r) {
    if (nv < 0 || nt < 0 || (nv > 0 && !xy) || (nt > 0 && !tri)) return GP_EINVAL;
    if (3ll * nt >= (1ll << 31)) return GP_ERANGE;
    hipStream_t s = c->stream;
    const size_t nxy = sizeof(int2) * (size_t)std::max(nv, 1), ntri = 12 * (size_t)std::max(nt, 1);
    const int32_t nmax = std::max(std::max(nv, nt), 1);
    const size_t sort = gp::renumber_sort_bytes(nmax);
    if (!sort) return GP_EHIP;
    int rc = c->pool.alloc(nxy, &r.xy);
    if (rc == GP_OK) rc = c->pool.alloc(ntri, &r.tri);
    if (rc == GP_OK) rc = c->pool.alloc(4 * (size_t)std::max(nv, 1), &r.vperm);
    if (rc == GP_OK) rc = c->pool.alloc(4 * (size_t)std::max(nt, 1), &r.tperm);
    const size_t tmp = arena_bytes<int32_t>(nmax) * 2 + arena_bytes<uint64_t>(nmax) * 2 + align_up(sort);
    if (rc == GP_OK) rc = c->pool.alloc(tmp, &r.tmp);
    const void *src_xy = xy, *src_tri = tri;
    if (rc == GP_OK && !in_dev) {   // the inputs are read several times: upload them once
        rc = c->pool.alloc(nxy, &r.in_xy);
        if (rc == GP_OK) rc = c->pool.alloc(ntri, &r.in_tri);
        if (rc == GP_OK &&
            ((nv > 0 && hipMemcpyAsync(r.in_xy, xy, sizeof(int2) * (size_t)nv, hipMemcpyHostToDevice, s) != hipSuccess) ||
             (nt > 0 && hipMemcpyAsync(r.in_tri, tri, 12 * (size_t)nt, hipMemcpyHostToDevice, s) != hipSuccess)))
            rc = GP_EHIP;
        src_xy = r.in_xy;
        src_tri = r.in_tri;
    }
    if (rc != GP_OK) {
        (void)hipGetLastError();
        return rc;
    }
    Arena a{static_cast<char *>(r.tmp), tmp, 0};
    gp::RenumberBuffers b{};
    b.xy_in = static_cast<const int2 *>(src_xy);
    b.tri_in = static_cast<const int32_t *>(src_tri);
    b.nv = nv;
    b.nt = nt;
    b.xy_out = static_cast<int2 *>(r.xy);
    b.tri_out = static_cast<int32_t *>(r.tri);
    b.vperm = static_cast<int32_t *>(r.vperm);
    b.tperm = static_cast<int32_t *>(r.tperm);
    b.vinv = a.take<int32_t>(nmax);
    b.vals = a.take<int32_t>(nmax);
    b.keys = a.take<uint64_t>(nmax);
    b.keys_alt = a.take<uint64_t>(nmax);
    b.sort_tmp = a.take<char>(sort);
    b.sort_bytes = sort;
    if (gp::launch_renumber(b, s) != hipSuccess) {
        (void)hipGetLastError();
        return GP_EHIP;
    }
    return GP_OK;
}

}  // namespace

// Builds meshes that each fit one workgroup with one launch of the small-job
// kernel in build-only mode: host inputs packed into one upload, the checks,
// orientation and twin matching in LDS (with the staged build's error codes
// and ranking), and one download of every mesh's error key and flip count.
int build_small_many(gp_ctx *c, int n, const int32_t *const *xy, const int32_t *nv, const int32_t *const *tri,
                     const int32_t *nt, uint32_t flags, gp_mesh **out, int *status) {
    const bool in_dev = (flags & GP_IN_DEVICE) != 0;
    std::vector<size_t> in_xy(n, 0), in_tri(n, 0);
    size_t in_bytes = 0;
    int max_nv = 0, max_nt = 0;
    for (int i = 0; i < n; i++) {
        out[i] = nullptr;
        status[i] = GP_OK;
        if (nv[i] < 0 || nt[i] < 0 || (nv[i] > 0 && !xy[i]) || (nt[i] > 0 && !tri[i])) status[i] = GP_EINVAL;
        if (status[i] != GP_OK) continue;
        max_nv = std::max(max_nv, nv[i]);
        max_nt = std::max(max_nt, nt[i]);
        if (in_dev) continue;
        in_xy[i] = in_bytes;
        in_bytes += align_up(8 * (size_t)nv[i], 16);
        in_tri[i] = in_bytes;
        in_bytes += align_up(12 * (size_t)nt[i], 16);
    }
    const size_t desc_off = align_up(in_bytes, 256), up_bytes = desc_off + sizeof(gp::SmallJob) * (size_t)n;
    const size_t cnt_off = align_up(up_bytes, 256), cnt_bytes = 4 * (size_t)gp::kJobCounts * (size_t)n;
    void *dev = nullptr;
    int rc = c->pool.alloc(cnt_off + cnt_bytes, &dev);
    char *up = rc == GP_OK ? static_cast<char *>(pinned_take(c, up_bytes)) : nullptr;
    char *down = up ? static_cast<char *>(pinned_take(c, cnt_bytes)) : nullptr;
    if (rc == GP_OK && (!up || !down)) rc = GP_ENOMEM;
    char *d = static_cast<char *>(dev);
    gp::SmallJob *descs = up ? reinterpret_cast<gp::SmallJob *>(up + desc_off) : nullptr;
    std::vector<gp_mesh *> ms(n, nullptr);
    for (int i = 0; i < n && rc == GP_OK; i++) {
        gp::SmallJob &sj = descs[i];
        sj = gp::SmallJob{};
        sj.counts = reinterpret_cast<int32_t *>(d + cnt_off) + (size_t)gp::kJobCounts * i;
        sj.build_only = 1;
        if (status[i] != GP_OK) continue;   // nothing to build: an empty job in the launch
        gp_mesh *m = new (std::nothrow) gp_mesh();
        if (!m) {
            status[i] = GP_ENOMEM;
            continue;
        }
        ms[i] = m;
        m->ctx = c;
        m->nv = nv[i];
        m->nt = nt[i];
        const size_t nh = 3 * (size_t)nt[i];
        void *p_xy = nullptr, *p_org = nullptr, *p_twin = nullptr;
        int r = c->pool.alloc(sizeof(int2) * std::max<size_t>(nv[i], 1), &p_xy);
        m->xy = static_cast<int2 *>(p_xy);
        if (r == GP_OK) r = c->pool.alloc(sizeof(int32_t) * std::max<size_t>(nh, 1), &p_org);
        m->org = static_cast<int32_t *>(p_org);
        if (r == GP_OK) r = c->pool.alloc(sizeof(int32_t) * std::max<size_t>(nh, 1), &p_twin);
        m->twin = static_cast<int32_t *>(p_twin);
        if (r != GP_OK) {
            status[i] = r;
            continue;
        }
        if (in_dev) {
            sj.xy = reinterpret_cast<const int2 *>(xy[i]);
            sj.tri = tri[i];
        } else {
            if (nv[i]) std::memcpy(up + in_xy[i], xy[i], 8 * (size_t)nv[i]);
            if (nt[i]) std::memcpy(up + in_tri[i], tri[i], 12 * (size_t)nt[i]);
            sj.xy = reinterpret_cast<const int2 *>(d + in_xy[i]);
            sj.tri = reinterpret_cast<const int32_t *>(d + in_tri[i]);
        }
        sj.nv = nv[i];
        sj.nt = nt[i];
        sj.org = m->org;
        sj.twin = m->twin;
        sj.xy_out = m->xy;
    }
    hipStream_t s = c->stream;
    if (rc == GP_OK &&
        (hipMemcpyAsync(d, up, up_bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
         gp::launch_small_jobs(reinterpret_cast<const gp::SmallJob *>(d + desc_off), n, max_nv, max_nt, s) !=
             hipSuccess ||
         hipMemcpyAsync(down, d + cnt_off, cnt_bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess)) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        rc = GP_EHIP;
    }
    for (int i = 0; i < n; i++) {
        gp_mesh *m = ms[i];
        if (!m) {
            if (rc != GP_OK && status[i] == GP_OK) status[i] = rc;
            continue;
        }
        int st = rc != GP_OK ? rc : status[i];
        if (st == GP_OK) {
            const int32_t *cnt = reinterpret_cast<const int32_t *>(down) + (size_t)gp::kJobCounts * i;
            const uint64_t key = (uint64_t)(uint32_t)cnt[8] | ((uint64_t)(uint32_t)cnt[9] << 32);
            if (key != ~0ull) {
                st = -(int)(key & 0xff);
            } else {
                m->nflipped = cnt[10];
                m->bytes = align_up(sizeof(int2) * (size_t)std::max(m->nv, 1)) +
                           2 * align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(3ll * m->nt, 1));
                if (flags & GP_COMPACT) st = compact_mesh(c, m, reinterpret_cast<int32_t *>(down) + (size_t)gp::kJobCounts * i);
            }
        }
        status[i] = st;
        if (st == GP_OK) {
            out[i] = m;
        } else {
            gpolylla_mesh_free(m);   // the stream has drained: nothing reads it
        }
    }
    if (up) pinned_give(c, up, up_bytes);
    if (down) pinned_give(c, down, cnt_bytes);
    if (dev) c->pool.release(dev);
    return GP_OK;
}

int build_many(gp_ctx *c, int n, const int32_t *const *xy, const int32_t *nv, const int32_t *const *tri,
               const int32_t *nt, uint32_t flags, gp_mesh **out, int *status) {
    if (!(flags & GP_RENUMBER) && n > 0 && n < 65536 && c->cfg.small_max > 0) {
        bool small = true;
        int max_nv = 0, max_nt = 0;
        for (int i = 0; i < n && small; i++) {
            small = nv[i] >= 0 && nt[i] >= 0 && nv[i] <= gp::kJobSmallV && nt[i] <= std::min(gp::kJobSmallTri, c->cfg.small_max);
            max_nv = std::max(max_nv, nv[i]);
            max_nt = std::max(max_nt, nt[i]);
        }
        if (small && gp::small_job_lds_bytes(max_nv, max_nt) <= (size_t)c->cfg.lds_max)
            return build_small_many(c, n, xy, nv, tri, nt, flags, out, status);
    }
    std::vector<BuildJob> jobs(n);
    const size_t hb = 16 * (size_t)std::max(n, 1);
    char *host = static_cast<char *>(pinned_take(c, hb));
    if (!host) return GP_ENOMEM;
    for (int i = 0; i < n; i++) {
        jobs[i].key_h = reinterpret_cast<unsigned long long *>(host + 16 * i);
        jobs[i].nflip_h = reinterpret_cast<int32_t *>(host + 16 * i + 8);
        out[i] = nullptr;
    }
    auto drain = [&]() {
        if (hipStreamSynchronize(c->stream) != hipSuccess) {
            (void)hipGetLastError();
            for (BuildJob &j : jobs)
                if (j.rc == GP_OK) j.rc = GP_EHIP;
        }
    };
    // renumbered inputs (GP_RENUMBER): built from their device copies
    std::vector<Renumbered> rn((flags & GP_RENUMBER) ? n : 0);
    for (int i = 0; i < n; i++) {
        if (flags & GP_RENUMBER) {
            jobs[i].rc = renumber_input(c, xy[i], nv[i], tri[i], nt[i], (flags & GP_IN_DEVICE) != 0, rn[i]);
            if (jobs[i].rc == GP_OK)
                jobs[i].rc = build_stage0(c, static_cast<const int32_t *>(rn[i].xy), nv[i],
                                          static_cast<const int32_t *>(rn[i].tri), nt[i], flags | GP_IN_DEVICE,
                                          jobs[i]);
        } else {
            jobs[i].rc = build_stage0(c, xy[i], nv[i], tri[i], nt[i], flags, jobs[i]);
        }
    }
    drain();
    for (BuildJob &j : jobs)
        if (j.rc == GP_OK) j.rc = build_stage1(c, j);
    drain();
    for (BuildJob &j : jobs)
        if (j.rc == GP_OK) j.rc = build_stage2(c, j);
    if (flags & GP_COMPACT)
        for (BuildJob &j : jobs)
            if (j.rc == GP_OK) j.rc = compact_mesh(c, j.m, j.nflip_h);
    // a failed job's memory goes back after the stream has drained its work
    // (as do the renumbered inputs, which the builds have finished reading)
    bool failed = false;
    for (BuildJob &j : jobs) failed |= j.rc != GP_OK;
    if (failed) drain();
    for (int i = 0; i < n; i++) {
        status[i] = jobs[i].rc;
        if (jobs[i].rc == GP_OK) {
            out[i] = jobs[i].m;
            if (!rn.empty()) {
                out[i]->vperm = static_cast<int32_t *>(rn[i].vperm);
                out[i]->tperm = static_cast<int32_t *>(rn[i].tperm);
                out[i]->bytes += align_up(4 * (size_t)std::max(nv[i], 1)) + align_up(4 * (size_t)std::max(nt[i], 1));
                renumbered_free(c, rn[i], true);
            }
        } else {
            build_abort(c, jobs[i]);
            if (!rn.empty()) renumbered_free(c, rn[i], false);
        }
    }
    pinned_give(c, host, hb);
    return GP_OK;
}

size_t build_footprint(int64_t nv, int64_t nt, bool inputs_on_device) {
    const int64_t nh = 3 * nt;
    const size_t keep = align_up(sizeof(int2) * (size_t)std::max<int64_t>(nv, 1)) +
                        2 * align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(nh, 1));
    const size_t tmp = arena_bytes<int32_t>(nv + 1) * 3 + arena_bytes<int2>(nh + 1) +
                       arena_bytes<uint64_t>(gp::build_scan_tiles((int32_t)nv)) + arena_bytes<int32_t>(4) +
                       arena_bytes<unsigned long long>(1) + (inputs_on_device ? 0 : arena_bytes<int32_t>(nh + 1));
    return keep + align_up(tmp);
}

size_t batch_footprint(const gp::LaunchCfg &cfg, const int32_t *nts, int n) {
    std::vector<gp::MeshDesc> descs(n);
    PlanSizes p;
    if (plan_core(cfg, nts, nullptr, n, descs.data(), &p) != GP_OK) return (size_t)-1;
    return align_up(p.out_bytes) + align_up(p.tmp_bytes);
}

}  // namespace gprt

namespace {

// A captured pipeline for one batch shape.  Its scratch (descriptor table,
// counters, lists, labels) stays allocated with it, so every kernel argument
// in the graph stays valid; per call only the descriptor table is rewritten
// (output pointers) before the replay.
struct GraphEntry {
    gp::LaunchCfg cfg;
    std::vector<int32_t> nts;
    bool compact = false;
    void *scratch = nullptr;
    gp::RunBuffers rb{};
    std::vector<uint8_t *> tflag, pl;
    std::vector<int32_t *> lpos;
    std::vector<gp::MeshDesc> staged;   // the descriptor table last staged into rb.descs
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

bool same_cfg(const gp::LaunchCfg &a, const gp::LaunchCfg &b) { return std::memcmp(&a, &b, sizeof a) == 0; }

}  // namespace

namespace gprt {
struct GraphCache {
    std::vector<GraphEntry> entries;
    uint64_t tick = 0;
};
}  // namespace gprt

namespace {

GraphCache &graphs_of(gp_ctx *c);

void graph_entry_free(gp_ctx *c, GraphEntry &e) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    c->pool.release(e.scratch);   // stream-ordered reuse
    e.exec = nullptr;
    e.scratch = nullptr;
}

int graph_entry(gp_ctx *c, const Plan &plan, GraphEntry **out) {
    GraphCache &gc = graphs_of(c);
    for (auto &e : gc.entries) {
        if (e.nts == plan.nts && e.compact == plan.compact && same_cfg(e.cfg, c->cfg)) {
            e.last_use = ++gc.tick;
            *out = &e;
            return GP_OK;
        }
    }
    if (gc.entries.size() >= 4) {   // evict the least recently used shape
        size_t k = 0;
        for (size_t i = 1; i < gc.entries.size(); i++)
            if (gc.entries[i].last_use < gc.entries[k].last_use) k = i;
        graph_entry_free(c, gc.entries[k]);
        gc.entries.erase(gc.entries.begin() + k);
    }
    GraphEntry e;
    e.cfg = c->cfg;
    e.nts = plan.nts;
    e.compact = plan.compact;
    int rc = c->pool.alloc(plan.tmp_bytes, &e.scratch);
    if (rc != GP_OK) return rc;
    const int n = (int)plan.nts.size();
    e.tflag.resize(n);
    e.pl.resize(n);
    e.lpos.resize(n);
    layout_scratch(plan, plan.descs.data(), n, e.scratch, &e.rb, e.tflag.data(), e.pl.data(), e.lpos.data());
    e.rb.compact = plan.compact;
    hipGraph_t graph = nullptr;
    hipStream_t s = c->stream;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        c->pool.release(e.scratch);
        return GP_EHIP;
    }
    hipError_t le = gp::launch_pipeline(c->cfg, e.rb, s, nullptr, nullptr);
    hipError_t ce = hipStreamEndCapture(s, &graph);
    if (le != hipSuccess || ce != hipSuccess || !graph ||
        hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        if (graph) (void)hipGraphDestroy(graph);
        c->pool.release(e.scratch);
        return GP_EHIP;
    }
    (void)hipGraphDestroy(graph);
    e.last_use = ++gc.tick;
    gc.entries.push_back(std::move(e));
    *out = &gc.entries.back();
    return GP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// scratch of gpolylla_mesh_noalloc: one static array per device
//
// In host code `scratch` names a host-side stand-in, not device memory; its
// device address is looked up once per device with hipGetSymbolAddress (at
// context creation, with the device current) and only that address is ever
// handed to kernels.
// ---------------------------------------------------------------------------

static __device__ __align__(256) char scratch[GP_NOALLOC_SCRATCH_BYTES];
static_assert(sizeof(gp_dev_counts) == 8 * sizeof(int32_t), "the counts kernel writes 8 int32");

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};

// Called with `device` current.  A failed lookup leaves the pointer null:
// contexts still work, gpolylla_mesh_noalloc then answers GP_EHIP.
void noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_tried[device]) return;
    g_scratch_tried[device] = true;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
    }
    g_scratch_ptr[device] = ptr;
}

void *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
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

namespace {

// Per-kernel launch shapes, "label=256x4,relink=256x2,compact=512x4,
// persist=1024x256" (any subset, any order; persist is blocks x threads of the
// list-driven kernels).  Every entry is checked; on any error *cfg is left as
// it was.  Tiles are then clamped to what each kernel's LDS staging allows.
int parse_launch_spec(const char *spec, gp::LaunchCfg *cfg) {
    gp::LaunchCfg g = *cfg;
    const std::string sp(spec);
    size_t p0 = 0;
    while (p0 < sp.size()) {
        size_t p1 = sp.find(',', p0);
        if (p1 == std::string::npos) p1 = sp.size();
        const std::string item = sp.substr(p0, p1 - p0);
        p0 = p1 + 1;
        const size_t eq = item.find('='), x = item.find('x', eq == std::string::npos ? 0 : eq);
        if (eq != std::string::npos && item.compare(0, eq, "small") == 0) {
            // small=N: meshes of at most N triangles run as one workgroup (0: never)
            const std::string sn = item.substr(eq + 1);
            if (sn.empty() || sn.size() > 6 || sn.find_first_not_of("0123456789") != std::string::npos)
                return GP_EINVAL;
            const int n = std::atoi(sn.c_str());
            if (n > gp::kSmallMaxTri) return GP_EINVAL;
            g.small_max = n;
            continue;
        }
        if (eq == std::string::npos || x == std::string::npos) return GP_EINVAL;
        const std::string k = item.substr(0, eq), sb = item.substr(eq + 1, x - eq - 1), si = item.substr(x + 1);
        if (sb.empty() || si.empty() || sb.size() > 6 || si.size() > 6 ||
            sb.find_first_not_of("0123456789") != std::string::npos ||
            si.find_first_not_of("0123456789") != std::string::npos)
            return GP_EINVAL;
        const int b = std::atoi(sb.c_str()), it = std::atoi(si.c_str());
        const bool ok_b = b >= 64 && b <= 1024 && b % 64 == 0;
        const bool ok_i = it == 1 || it == 2 || it == 4 || it == 8;
        if (k == "persist") {
            if (!ok_b || it < 1 || it > 65536) return GP_EINVAL;
            g.block_persistent = b;
            g.persistent_blocks = it;
        } else if (!ok_b || !ok_i) {
            return GP_EINVAL;
        } else if (k == "label") {
            g.block_label = b;
            g.items_label = it;
        } else if (k == "relink") {
            g.block_relink = b;
            g.items_relink = it;
        } else if (k == "compact") {
            g.block_compact = b;
            g.items_compact = it;
        } else {
            return GP_EINVAL;
        }
    }
    // LDS per tile: k_label stages 12 bytes per triangle (tile <= 4096),
    // k_relink 19 bytes (tile <= 1024), k_compact 19 bytes (tile <= 2048)
    while ((int64_t)g.block_label * g.items_label > 4096 && g.items_label > 1) g.items_label /= 2;
    while ((int64_t)g.block_relink * g.items_relink > 1024 && g.items_relink > 1) g.items_relink /= 2;
    while ((int64_t)g.block_compact * g.items_compact > 2048 && g.items_compact > 1) g.items_compact /= 2;
    *cfg = g;
    return GP_OK;
}

// Dynamic LDS one k_small workgroup may use on a device (the current one),
// from the device's per-workgroup limit; looked up once per device.
int small_lds_limit(int device) {
    static std::mutex mu;
    static int limit[kMaxDevices];
    static bool known[kMaxDevices];
    std::lock_guard<std::mutex> lk(mu);
    if (device < 0 || device >= kMaxDevices) return 0;
    if (!known[device]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess || v < 0) {
            (void)hipGetLastError();
            v = 0;
        }
        limit[device] = v > 0 ? gp::prepare_small(v) : 0;
        known[device] = true;
    }
    return limit[device];
}

}  // namespace

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
    noalloc_setup(device);
    c->cfg.lds_max = small_lds_limit(device);
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
    (void)parse_launch_spec("", &c->cfg);   // clamps the tiles of opts->block x opts->items
    if (const char *env = std::getenv("GPOLYLLA_CFG"))
        (void)parse_launch_spec(env, &c->cfg);   // launch shapes from the environment; ignored if malformed
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
    if (c->graphs) {
        for (auto &e : c->graphs->entries) graph_entry_free(c, e);
        delete c->graphs;
        c->graphs = nullptr;
    }
    for (auto e : c->spare_events) (void)hipEventDestroy(e);
    for (auto e : c->done_events) (void)hipEventDestroy(e);
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

int gpolylla_ctx_set_debug(gp_ctx *c, int32_t on) {
    if (!c) return GP_EINVAL;
    c->debug = on != 0;
    return GP_OK;
}

int gpolylla_result_debug(gp_result *x, gp_result_debug *out) {
    if (!x || !out || !x->run || x->host) return GP_EINVAL;
    RunState *r = x->run;
    if (!r->dbg) return GP_EINVAL;   // not a debug run
    const int st = run_sync(r);
    if (st != GP_OK && st != GP_ECORRUPT) return st;
    DeviceGuard g(r->ctx->device);
    const DebugSnap &d = *r->dbg;
    const int i = x->index;
    const size_t nt = (size_t)x->nt, nh = 3 * nt;
    if (nt && out->tflag_relink) HIP_OK(hipMemcpy(out->tflag_relink, d.tflag_relink[i], nt, hipMemcpyDeviceToHost));
    if (nt && out->tflag_final) HIP_OK(hipMemcpy(out->tflag_final, d.tflag_final[i], nt, hipMemcpyDeviceToHost));
    if (nh && out->next_relink) HIP_OK(hipMemcpy(out->next_relink, d.next_relink[i], 4 * nh, hipMemcpyDeviceToHost));
    if (nh && out->prev_relink) HIP_OK(hipMemcpy(out->prev_relink, d.prev_relink[i], 4 * nh, hipMemcpyDeviceToHost));
    int32_t total = 0;
    HIP_OK(hipMemcpy(&total, d.ntips, sizeof total, hipMemcpyDeviceToHost));
    total = std::max(0, std::min(total, d.cap_tips));
    std::vector<gp::ListEntry> all((size_t)total);
    if (total) HIP_OK(hipMemcpy(all.data(), d.tips, sizeof(gp::ListEntry) * (size_t)total, hipMemcpyDeviceToHost));
    int32_t k = 0;
    for (const gp::ListEntry &e : all) {
        if (e.mesh != i) continue;
        if (out->tips && k < out->tips_cap) out->tips[k] = e.he;
        k++;
    }
    out->ntips = k;
    return st;
}

void gpolylla_ctx_kernel_reset(gp_ctx *c) {
    if (!c) return;
    for (int k = 0; k < gp::K_COUNT; k++) {
        c->kms[k] = 0;
        c->kcount[k] = 0;
    }
}

int gpolylla_ctx_set_launch(gp_ctx *c, const char *spec) {
    if (!c || !spec) return GP_EINVAL;
    return parse_launch_spec(spec, &c->cfg);
}

int gpolylla_ctx_get_launch(const gp_ctx *c, char *buf, int32_t cap) {
    if (!c) return GP_EINVAL;
    const gp::LaunchCfg &g = c->cfg;
    char tmp[192];
    const int n = std::snprintf(tmp, sizeof tmp, "label=%dx%d,relink=%dx%d,compact=%dx%d,persist=%dx%d,small=%d",
                                g.block_label, g.items_label, g.block_relink, g.items_relink, g.block_compact,
                                g.items_compact, g.block_persistent, g.persistent_blocks, g.small_max);
    if (buf && cap > 0) {
        const int m = n < cap - 1 ? n : cap - 1;
        std::memcpy(buf, tmp, (size_t)m);
        buf[m] = 0;
    }
    return n + 1;
}

// ---------------------------------------------------------------------------
// build
// ---------------------------------------------------------------------------

int gpolylla_build_halfedges(gp_ctx *c, const int32_t *xy, int32_t nv, const int32_t *tri, int32_t nt,
                             uint32_t flags, gp_mesh **out) {
    if (!c || !out) return GP_EINVAL;
    *out = nullptr;
    DeviceGuard g(c->device);
    gp_mesh *m = nullptr;
    int st = GP_OK;
    const int rc = gprt::build_many(c, 1, &xy, &nv, &tri, &nt, flags, &m, &st);
    if (rc != GP_OK) return rc;
    if (st != GP_OK) return st;
    *out = m;
    return GP_OK;
}

int gpolylla_mesh_copy(const gp_mesh *m, int32_t *org, int32_t *twin, int64_t *nflipped) {
    if (!m) return GP_EINVAL;
    DeviceGuard g(m->ctx->device);
    size_t n = sizeof(int32_t) * 3 * (size_t)m->nt;
    if (nflipped) *nflipped = m->nflipped;
    if (!n || (!org && !twin)) return GP_OK;
    if (!m->org8) {
        if (org) HIP_OK(hipMemcpy(org, m->org, n, hipMemcpyDeviceToHost));
        if (twin) HIP_OK(hipMemcpy(twin, m->twin, n, hipMemcpyDeviceToHost));
        return GP_OK;
    }
    // a compact mesh: decode into scratch first
    gp_ctx *c = m->ctx;
    void *p = nullptr;
    int rc = c->pool.alloc(2 * align_up(n), &p);
    if (rc != GP_OK) return rc;
    int32_t *dorg = static_cast<int32_t *>(p);
    int32_t *dtwin = reinterpret_cast<int32_t *>(static_cast<char *>(p) + align_up(n));
    gp::CompactBuffers cb{};
    cb.nt = m->nt;
    cb.org8 = m->org8;
    cb.twin16 = m->twin16;
    cb.esc = m->esc;
    cb.esc_mask = m->esc_mask;
    if (gp::launch_compact_decode(cb, dorg, dtwin, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess ||
        (org && hipMemcpy(org, dorg, n, hipMemcpyDeviceToHost) != hipSuccess) ||
        (twin && hipMemcpy(twin, dtwin, n, hipMemcpyDeviceToHost) != hipSuccess)) {
        (void)hipGetLastError();
        rc = GP_EHIP;
    }
    c->pool.release(p);
    return rc;
}

int gpolylla_mesh_permutation(const gp_mesh *m, int32_t *tri_new_to_old, int32_t *vert_new_to_old) {
    if (!m || !m->tperm) return GP_EINVAL;
    DeviceGuard g(m->ctx->device);
    if (tri_new_to_old && m->nt)
        HIP_OK(hipMemcpy(tri_new_to_old, m->tperm, 4 * (size_t)m->nt, hipMemcpyDeviceToHost));
    if (vert_new_to_old && m->nv)
        HIP_OK(hipMemcpy(vert_new_to_old, m->vperm, 4 * (size_t)m->nv, hipMemcpyDeviceToHost));
    return GP_OK;
}

int gpolylla_mesh_bytes(const gp_mesh *m, size_t *bytes, int64_t *escapes) {
    if (!m) return GP_EINVAL;
    if (bytes) *bytes = m->bytes;
    if (escapes) *escapes = m->nesc;
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
    m->ctx->pool.release(m->org8);
    m->ctx->pool.release(m->twin16);
    m->ctx->pool.release(m->esc);
    m->ctx->pool.release(m->vperm);
    m->ctx->pool.release(m->tperm);
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
    Plan plan;
    int rc = make_plan(c->cfg, meshes, n, &plan);
    if (rc != GP_OK) return rc;
    reap_retired(c, false);

    // one small mesh runs as one kernel launch with its descriptor as the
    // argument and its counts written straight to host memory: no scratch,
    // nothing staged, no graph (there is one kernel to launch)
    const bool small_one = n == 1 && !c->profile && !c->debug && gp::small_fits(c->cfg, meshes[0]->nt);
    // scratch: per call from the pool, or owned by a cached graph
    const bool use_graph = (out_flags & GP_GRAPH) && !c->profile && !c->debug && !small_one;
    GraphEntry *ge = nullptr;
    void *p_tmp = nullptr;
    if (use_graph) {
        rc = graph_entry(c, plan, &ge);
        if (rc != GP_OK) return rc;
    } else if (!small_one) {
        rc = c->pool.alloc(plan.tmp_bytes, &p_tmp);
        if (rc != GP_OK) return rc;
    }
    RunState *r = new (std::nothrow) RunState();
    if (!r) {
        c->pool.release(p_tmp);
        return GP_ENOMEM;
    }
    r->ctx = c;
    r->nmesh = n;
    rc = c->pool.alloc(plan.out_bytes, &r->out_block);
    if (rc == GP_OK) {
        r->host_ctrs_bytes = sizeof(gp::MeshCounters) * n;
        r->host_ctrs = static_cast<gp::MeshCounters *>(pinned_take(c, r->host_ctrs_bytes));
        if (!r->host_ctrs) rc = GP_ENOMEM;
    }
    if (rc == GP_OK && !c->done_events.empty()) {
        r->done = c->done_events.back();
        c->done_events.pop_back();
    } else if (rc == GP_OK && hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess) {
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
    gp::RunBuffers rb{};
    std::vector<uint8_t *> tflag(n), pl(n);
    std::vector<int32_t *> lpos(n);
    if (ge) {
        rb = ge->rb;
        tflag = ge->tflag;
        pl = ge->pl;
        lpos = ge->lpos;
    } else if (!small_one) {
        layout_scratch(plan, plan.descs.data(), n, p_tmp, &rb, tflag.data(), pl.data(), lpos.data());
        rb.compact = plan.compact;
        rb.chain_only = c->debug;   // the snapshots are of the chain's intermediate stages
    }
    Arena ao{static_cast<char *>(r->out_block), plan.out_bytes, 0};
    std::vector<gp_result *> res(n, nullptr);
    std::vector<gp::MeshDesc> descs = plan.descs;
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
        mesh_desc_fill(m, d);
        d.next_o = x->next_o;
        d.prev_o = x->prev_o;
        d.seeds = x->seeds;
        d.loop_off = x->loop_off;
        d.loop_he = x->loop_he;
        d.tflag = tflag[i];
        d.pl = pl[i];
        d.lpos = lpos[i];
        d.ctr = small_one ? nullptr : rb.ctrs + i;
    }
    hipStream_t s = c->stream;
    int err = GP_OK;
    // a captured graph keeps its descriptor table; it is staged again only
    // when it changed (when the pool hands back the same output block, as it
    // does when results are freed between calls, it has not)
    const size_t dbytes = sizeof(gp::MeshDesc) * n;
    const bool same = ge && ge->staged.size() == descs.size() &&
                      std::memcmp(ge->staged.data(), descs.data(), dbytes) == 0;
    if (!same && !small_one) {
        if (stage_to_device(c, const_cast<gp::MeshDesc *>(rb.descs), descs.data(), dbytes) != hipSuccess)
            err = GP_EHIP;
        else if (ge)
            ge->staged = descs;
    }
    DebugHook dh{c, nullptr, &rb, &res, &tflag};
    if (err == GP_OK && c->debug) {
        // the snapshots' memory: per mesh two label arrays and next', prev'
        DebugSnap *d = new (std::nothrow) DebugSnap();
        size_t bytes = align_up(sizeof(gp::ListEntry) * (size_t)std::max(rb.cap_tips, 1)) + kAlign;
        for (int i = 0; i < n; i++)
            bytes += 2 * align_up((size_t)std::max(res[i]->nt, 1)) +
                     2 * align_up(sizeof(int32_t) * 3 * (size_t)std::max(res[i]->nt, 1));
        if (!d || c->pool.alloc(bytes, &d->block) != GP_OK) {
            delete d;
            err = GP_ENOMEM;
        } else {
            Arena ad{static_cast<char *>(d->block), bytes, 0};
            d->cap_tips = rb.cap_tips;
            d->tips = ad.take<gp::ListEntry>((size_t)std::max(rb.cap_tips, 1));
            d->ntips = ad.take<int32_t>(1);
            for (int i = 0; i < n; i++) {
                const size_t nt = (size_t)std::max(res[i]->nt, 1);
                d->tflag_relink.push_back(ad.take<uint8_t>(nt));
                d->tflag_final.push_back(ad.take<uint8_t>(nt));
                d->next_relink.push_back(ad.take<int32_t>(3 * nt));
                d->prev_relink.push_back(ad.take<int32_t>(3 * nt));
            }
            r->dbg = d;
            dh.d = d;
        }
    }
    if (err == GP_OK) {
        hipError_t e = small_one ? gp::launch_small_one(descs[0], r->host_ctrs, s)
                       : ge      ? hipGraphLaunch(ge->exec, s)
                       : c->debug ? gp::launch_pipeline(c->cfg, rb, s, debug_hook, &dh)
                                  : gp::launch_pipeline(c->cfg, rb, s, c->profile ? profile_hook : nullptr, c);
        if (e != hipSuccess) err = GP_EHIP;
    }
    if (err == GP_OK && !small_one &&
        gp::launch_copy_words(r->host_ctrs, rb.ctrs, sizeof(gp::MeshCounters) * n, s) != hipSuccess)
        err = GP_EHIP;
    if (err == GP_OK && hipEventRecord(r->done, s) != hipSuccess) err = GP_EHIP;
    // per-call temporaries go back to the pool; later users are ordered after
    // this run on the same stream
    c->pool.release(p_tmp);
    if (err != GP_OK) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        for (auto q : res) delete q;
        c->pool.release(r->out_block);
        if (r->dbg) c->pool.release(r->dbg->block);
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

namespace {
GraphCache &graphs_of(gp_ctx *c) {
    if (!c->graphs) c->graphs = new GraphCache();
    return *c->graphs;
}
}  // namespace

int gpolylla_mesh(gp_ctx *c, const gp_mesh *m, uint32_t out_flags, gp_result **out) {
    if (!m) return GP_EINVAL;
    return gpolylla_mesh_batch(c, &m, 1, out_flags, out);
}

int gpolylla_mesh_noalloc(gp_ctx *c, const gp_mesh *m, const gp_result_dev *out, gp_dev_counts *counts) {
    if (!c || !m || !out || !counts || m->ctx != c) return GP_EINVAL;
    if (!out->next || !out->prev || !out->seeds || !out->loop_off || !out->loop_he) return GP_EINVAL;
    void *base = noalloc_scratch(c->device);
    if (!base) return GP_EHIP;
    // one mesh: the plan fits on the stack, nothing is allocated anywhere
    gp::MeshDesc d;
    PlanSizes plan;
    int rc = plan_core(c->cfg, &m->nt, &m->nv, 1, &d, &plan);
    if (rc != GP_OK) return rc;
    if (plan.tmp_bytes > GP_NOALLOC_SCRATCH_BYTES) return GP_ETOOBIG;
    DeviceGuard g(c->device);
    gp::RunBuffers rb;
    uint8_t *tflag = nullptr, *pl = nullptr;
    int32_t *lpos = nullptr;
    layout_scratch(plan, &d, 1, base, &rb, &tflag, &pl, &lpos);
    rb.compact = m->org8 != nullptr;
    mesh_desc_fill(m, d);
    d.next_o = out->next;
    d.prev_o = out->prev;
    d.seeds = out->seeds;
    d.loop_off = out->loop_off;
    d.loop_he = out->loop_he;
    d.tflag = tflag;
    d.pl = pl;
    d.lpos = lpos;
    d.ctr = rb.ctrs;
    hipStream_t s = c->stream;
    // every counter and list the kernels use is cleared by the chain itself
    // (no memset node, so the call can be captured into a graph)
    if (gp::launch_put_desc(d, const_cast<gp::MeshDesc *>(rb.descs), s) != hipSuccess ||
        gp::launch_pipeline(c->cfg, rb, s, nullptr, nullptr) != hipSuccess ||
        gp::launch_export_counts(rb.ctrs, reinterpret_cast<int32_t *>(counts), s) != hipSuccess) {
        (void)hipGetLastError();
        return GP_EHIP;
    }
    return GP_OK;
}

int gpolylla_result_info(gp_result *x, gp_result_info *info) {
    if (x && info && x->host) {
        *info = x->hinfo;
        return GP_OK;
    }
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
    info->loops_only = 0;
    return GP_OK;
}

int gpolylla_result_copy(gp_result *x, int32_t *next, int32_t *prev, int32_t *seeds, int32_t *loop_off,
                         int32_t *loop_he) {
    gp_result_info info;
    int st = gpolylla_result_info(x, &info);
    if (st != GP_OK) return st;
    if (x->host) {
        const size_t nh = (size_t)info.nh;
        if ((next || prev) && info.loops_only) return GP_EINVAL;
        if (next && nh) std::memcpy(next, x->next_o, 4 * nh);
        if (prev && nh) std::memcpy(prev, x->prev_o, 4 * nh);
        if (seeds && info.npoly) std::memcpy(seeds, x->seeds, 4 * (size_t)info.npoly);
        if (loop_off) std::memcpy(loop_off, x->loop_off, 4 * (size_t)(info.npoly + 1));
        if (loop_he && info.nloop_he) std::memcpy(loop_he, x->loop_he, 4 * (size_t)info.nloop_he);
        return GP_OK;
    }
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
    if (!x || !dev || !x->run || x->host) return GP_EINVAL;
    dev->next = x->next_o;
    dev->prev = x->prev_o;
    dev->seeds = x->seeds;
    dev->loop_off = x->loop_off;
    dev->loop_he = x->loop_he;
    return GP_OK;
}

void gpolylla_result_free(gp_result *x) {
    if (!x) return;
    if (x->host) {
        if (x->on_free) x->on_free();
    } else {
        run_unref(x->run);
    }
    delete x;
}

}  // extern "C"
