// gpolylla_mesh_jobs: meshes a list of host-resident triangulations with the
// host<->device copies of one group of jobs overlapped with the copies and
// the work of the next.
//
// One host thread and three streams: an upload stream, the context's stream
// (builds and meshing runs, in job order) and a download stream.  Per group
// of jobs (consecutive jobs up to a triangle budget, meshed as one batch):
//   1. queue the uploads of the next group's inputs;
//   2. wait for the previous group's meshing run to finish and queue its
//      downloads, so they run while this group builds and the next uploads;
//   3. build this group's half-edge structures (after its uploads; two host
//      checks for the whole group) and queue its meshing run;
//   4. give back the memory of groups whose downloads have completed (at
//      most two meshed groups hold memory at once).
// Memory goes back to the context's pool only after the host has seen the
// downloads that read it complete, so the pool's reuse stays ordered.
#include <algorithm>
#include <cstring>
#include <deque>
#include <vector>

#include "runtime_internal.h"

using namespace gprt;

namespace {

struct Group {
    int j0 = 0, j1 = 0;                // jobs [j0, j1)
    std::vector<void *> dxy, dtri;     // uploaded inputs (until the builds)
    hipEvent_t uploaded = nullptr;     // the uploads have finished
    int up_rc = GP_OK;
    std::vector<int> job;              // job of each meshed entry
    std::vector<gp_mesh *> meshes;
    std::vector<gp_result *> res;
    hipEvent_t copied = nullptr;       // the group's downloads have finished
    bool queued = false;               // downloads queued
};

void group_free(Group &g) {
    for (gp_result *r : g.res) gpolylla_result_free(r);
    for (gp_mesh *m : g.meshes) gpolylla_mesh_free(m);
    g.res.clear();
    g.meshes.clear();
    if (g.copied) (void)hipEventDestroy(g.copied);
    g.copied = nullptr;
    if (g.uploaded) (void)hipEventDestroy(g.uploaded);
    g.uploaded = nullptr;
}

// Waits for the group's meshing run and queues the downloads of every job's
// outputs on the copy stream.
void group_download(gp_job *jobs, Group &g, hipStream_t cs) {
    for (size_t k = 0; k < g.res.size(); k++) {
        gp_job &jb = jobs[g.job[k]];
        gp_result_info info;
        int rc = gpolylla_result_info(g.res[k], &info);   // waits for the run
        gp_result_dev dv{};
        if (rc == GP_OK) rc = gpolylla_result_device(g.res[k], &dv);
        if (rc == GP_OK) {
            jb.npoly = info.npoly;
            jb.nloop_he = info.nloop_he;
            const size_t nh = (size_t)info.nh, P = (size_t)info.npoly, F = (size_t)info.nloop_he;
            hipError_t e = hipSuccess;
            if (jb.next && nh) e = hipMemcpyAsync(jb.next, dv.next, 4 * nh, hipMemcpyDeviceToHost, cs);
            if (e == hipSuccess && jb.prev && nh)
                e = hipMemcpyAsync(jb.prev, dv.prev, 4 * nh, hipMemcpyDeviceToHost, cs);
            if (e == hipSuccess && P) e = hipMemcpyAsync(jb.seeds, dv.seeds, 4 * P, hipMemcpyDeviceToHost, cs);
            if (e == hipSuccess)
                e = hipMemcpyAsync(jb.loop_off, dv.loop_off, 4 * (P + 1), hipMemcpyDeviceToHost, cs);
            if (e == hipSuccess && F) e = hipMemcpyAsync(jb.loop_he, dv.loop_he, 4 * F, hipMemcpyDeviceToHost, cs);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                rc = GP_EHIP;
            }
        }
        jb.status = rc;
    }
    if (hipEventCreateWithFlags(&g.copied, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(g.copied, cs) != hipSuccess) {
        (void)hipGetLastError();
        if (g.copied) (void)hipEventDestroy(g.copied);
        g.copied = nullptr;
        (void)hipStreamSynchronize(cs);   // without the event: wait here
    }
    g.queued = true;
}

// Waits for the group's downloads, then frees its device memory.
void group_finish(Group &g, hipStream_t cs) {
    if (!g.copied || hipEventSynchronize(g.copied) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(cs);
    }
    group_free(g);
}

// ---- small jobs: packed copies, one build-and-mesh launch per group -------
//
// A list whose jobs all fit one workgroup (gp::kJobSmallTri triangles,
// gp::kJobSmallV vertices) is not worth a build and a batched run per group:
// the dozen runtime calls per job that those take would bound it.  Each
// group's inputs are packed into one pinned staging block and uploaded with
// one copy; one launch builds and meshes every job (k_small_jobs); one copy
// brings every output back, and the host hands each job its part.

bool small_jobs_fit(const gp_ctx *c, const gp_job *jobs, int n) {
    int max_nv = 0, max_nt = 0;
    for (int i = 0; i < n; i++) {
        if (jobs[i].nt > gp::kJobSmallTri || jobs[i].nv > gp::kJobSmallV) return false;
        max_nv = std::max(max_nv, jobs[i].nv);
        max_nt = std::max(max_nt, jobs[i].nt);
    }
    return c->cfg.small_max >= max_nt && gp::small_job_lds_bytes(max_nv, max_nt) <= (size_t)c->cfg.lds_max;
}

// Byte offsets of one job's parts: inputs (xy, tri) in the upload block;
// structure scratch (org, twin) and outputs (counts, next, prev, seeds,
// loop_off, loop_he) in the device block, outputs contiguous per group.
struct SmallLayout {
    size_t xy, tri, org, twin, counts, next, prev, seeds, loop_off, loop_he;
};

// One packed group in flight: its layout, staging blocks and device block.
struct SmallGroup {
    int j0 = 0, j1 = 0;
    std::vector<SmallLayout> lay;
    char *up = nullptr, *down = nullptr;
    size_t up_bytes = 0, out_bytes = 0;
    void *dev = nullptr;
    hipEvent_t done = nullptr;
    int rc = GP_OK;
};

// Packs jobs [j0, j1) and queues their upload, the launch and the download.
void small_group_start(gp_ctx *c, gp_job *jobs, SmallGroup &g) {
    const int n = g.j1 - g.j0;
    g.lay.assign(n, SmallLayout{});
    size_t in_bytes = 0, scratch_bytes = 0, out_bytes = 0;
    int max_nv = 0, max_nt = 0;
    for (int k = 0; k < n; k++) {
        const gp_job &jb = jobs[g.j0 + k];
        const size_t nh = 3 * (size_t)jb.nt;
        SmallLayout &L = g.lay[k];
        L.xy = in_bytes;
        in_bytes += align_up(8 * (size_t)jb.nv, 16);
        L.tri = in_bytes;
        in_bytes += align_up(12 * (size_t)jb.nt, 16);
        L.org = scratch_bytes;
        scratch_bytes += align_up(4 * nh + 4, 16);
        L.twin = scratch_bytes;
        scratch_bytes += align_up(4 * nh + 4, 16);
        L.counts = out_bytes;
        out_bytes += align_up(4 * (size_t)gp::kJobCounts, 16);
        L.next = out_bytes;
        out_bytes += align_up(4 * nh + 4, 16);
        L.prev = out_bytes;
        out_bytes += align_up(4 * nh + 4, 16);
        L.seeds = out_bytes;
        out_bytes += align_up(4 * (size_t)jb.nt + 4, 16);
        L.loop_off = out_bytes;
        out_bytes += align_up(4 * (size_t)jb.nt + 8, 16);
        L.loop_he = out_bytes;
        out_bytes += align_up(4 * nh + 4, 16);
        max_nv = std::max(max_nv, jb.nv);
        max_nt = std::max(max_nt, jb.nt);
    }
    const size_t desc_off = align_up(in_bytes, 256);
    g.up_bytes = desc_off + sizeof(gp::SmallJob) * (size_t)n;   // inputs, then descriptors
    g.out_bytes = out_bytes;
    const size_t scratch_off = align_up(g.up_bytes, 256), out_off = align_up(scratch_off + scratch_bytes, 256);
    g.rc = c->pool.alloc(out_off + out_bytes, &g.dev);
    if (g.rc != GP_OK) return;
    g.up = static_cast<char *>(pinned_take(c, g.up_bytes));
    g.down = static_cast<char *>(pinned_take(c, g.out_bytes));
    if (!g.up || !g.down || hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        g.rc = GP_ENOMEM;
        return;
    }
    char *d = static_cast<char *>(g.dev);
    gp::SmallJob *descs = reinterpret_cast<gp::SmallJob *>(g.up + desc_off);
    for (int k = 0; k < n; k++) {
        const gp_job &jb = jobs[g.j0 + k];
        const SmallLayout &L = g.lay[k];
        if (jb.nv) std::memcpy(g.up + L.xy, jb.xy, 8 * (size_t)jb.nv);
        if (jb.nt) std::memcpy(g.up + L.tri, jb.tri, 12 * (size_t)jb.nt);
        gp::SmallJob &sj = descs[k];
        sj.xy = reinterpret_cast<const int2 *>(d + L.xy);
        sj.tri = reinterpret_cast<const int32_t *>(d + L.tri);
        sj.nv = jb.nv;
        sj.nt = jb.nt;
        sj.org = reinterpret_cast<int32_t *>(d + scratch_off + L.org);
        sj.twin = reinterpret_cast<int32_t *>(d + scratch_off + L.twin);
        sj.counts = reinterpret_cast<int32_t *>(d + out_off + L.counts);
        sj.next_o = reinterpret_cast<int32_t *>(d + out_off + L.next);
        sj.prev_o = reinterpret_cast<int32_t *>(d + out_off + L.prev);
        sj.seeds = reinterpret_cast<int32_t *>(d + out_off + L.seeds);
        sj.loop_off = reinterpret_cast<int32_t *>(d + out_off + L.loop_off);
        sj.loop_he = reinterpret_cast<int32_t *>(d + out_off + L.loop_he);
        sj.xy_out = nullptr;
        sj.build_only = 0;
        sj.pad = 0;
    }
    hipStream_t s = c->stream;
    if (hipMemcpyAsync(d, g.up, g.up_bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
        gp::launch_small_jobs(reinterpret_cast<const gp::SmallJob *>(d + desc_off), n, max_nv, max_nt, s) !=
            hipSuccess ||
        hipMemcpyAsync(g.down, d + out_off, g.out_bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipEventRecord(g.done, s) != hipSuccess) {
        (void)hipGetLastError();
        g.rc = GP_EHIP;
    }
}

// Waits for a started group, hands each job its outputs and status, and
// gives the group's memory back.
void small_group_finish(gp_ctx *c, gp_job *jobs, SmallGroup &g) {
    if (g.rc == GP_OK && hipEventSynchronize(g.done) != hipSuccess) {
        (void)hipGetLastError();
        g.rc = GP_EHIP;
    }
    if (g.rc != GP_OK) (void)hipStreamSynchronize(c->stream);   // nothing may still read or write the blocks
    for (int k = 0; k < g.j1 - g.j0 && g.rc == GP_OK; k++) {
        gp_job &jb = jobs[g.j0 + k];
        const SmallLayout &L = g.lay[k];
        const int32_t *cnt = reinterpret_cast<const int32_t *>(g.down + L.counts);
        const uint64_t key = (uint64_t)(uint32_t)cnt[8] | ((uint64_t)(uint32_t)cnt[9] << 32);
        gp::MeshCounters mc;
        std::memcpy(&mc, cnt, sizeof mc);
        if (key != ~0ull) {
            jb.status = -(int)(key & 0xff);
            continue;
        }
        if (mc.err || mc.npoly < 0 || mc.npoly > jb.nt || mc.nloop < 0 || mc.nloop > 3 * jb.nt) {
            jb.status = GP_ECORRUPT;
            continue;
        }
        const size_t nh = 3 * (size_t)jb.nt;
        jb.npoly = mc.npoly;
        jb.nloop_he = mc.nloop;
        if (jb.next && nh) std::memcpy(jb.next, g.down + L.next, 4 * nh);
        if (jb.prev && nh) std::memcpy(jb.prev, g.down + L.prev, 4 * nh);
        if (mc.npoly) std::memcpy(jb.seeds, g.down + L.seeds, 4 * (size_t)mc.npoly);
        std::memcpy(jb.loop_off, g.down + L.loop_off, 4 * ((size_t)mc.npoly + 1));
        if (mc.nloop) std::memcpy(jb.loop_he, g.down + L.loop_he, 4 * (size_t)mc.nloop);
        jb.status = GP_OK;
    }
    if (g.rc != GP_OK)
        for (int k = g.j0; k < g.j1; k++) jobs[k].status = g.rc;
    if (g.up) pinned_give(c, g.up, g.up_bytes);
    if (g.down) pinned_give(c, g.down, g.out_bytes);
    if (g.dev) c->pool.release(g.dev);
    if (g.done) (void)hipEventDestroy(g.done);
    g = SmallGroup{};
}

}  // namespace

extern "C" {

int gpolylla_mesh_jobs(gp_ctx *c, gp_job *jobs, int32_t n, int64_t group_triangles, uint32_t flags) {
    if (!c || n < 0 || (n > 0 && !jobs)) return GP_EINVAL;
    if (flags & ~(uint32_t)GP_GRAPH) return GP_EINVAL;
    for (int i = 0; i < n; i++) {
        const gp_job &j = jobs[i];
        if (j.nv < 0 || j.nt < 0 || (j.nv > 0 && !j.xy) || (j.nt > 0 && !j.tri) || !j.seeds || !j.loop_off ||
            !j.loop_he || ((j.next == nullptr) != (j.prev == nullptr)))
            return GP_EINVAL;
        if (3ll * j.nt >= (1ll << 31)) return GP_ERANGE;
    }
    for (int i = 0; i < n; i++) {
        jobs[i].npoly = jobs[i].nloop_he = 0;
        jobs[i].status = GP_OK;
    }
    if (n == 0) return GP_OK;
    const int64_t budget = group_triangles > 0 ? group_triangles : ((int64_t)8 << 20);
    DeviceGuard dg(c->device);
    if (small_jobs_fit(c, jobs, n)) {   // every job builds and meshes in one workgroup
        // two groups in flight: the host packs the next while the device
        // works on the current one, and unpacks it while the next runs
        SmallGroup cur, nxt;
        int j0 = 0;
        auto form = [&](SmallGroup &g) {
            int64_t tri = 0;
            g.j0 = g.j1 = j0;
            while (g.j1 < n && g.j1 - g.j0 < 65535 && (g.j1 == g.j0 || tri + jobs[g.j1].nt <= budget))
                tri += jobs[g.j1++].nt;
            j0 = g.j1;
            small_group_start(c, jobs, g);
        };
        form(cur);
        while (true) {
            const bool more = j0 < n;
            if (more) form(nxt);
            small_group_finish(c, jobs, cur);
            if (!more) break;
            cur = std::move(nxt);
            nxt = SmallGroup{};
        }
        int rc_all = GP_OK;
        for (int i = 0; i < n; i++)
            if (jobs[i].status != GP_OK && rc_all == GP_OK) rc_all = jobs[i].status;
        return rc_all;
    }
    hipStream_t us = nullptr, cs = nullptr;   // uploads, downloads
    if (hipStreamCreateWithFlags(&us, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        if (us) (void)hipStreamDestroy(us);
        return GP_EHIP;
    }
    hipStream_t s = c->stream;
    const uint32_t mesh_flags = GP_ASYNC | (flags & GP_GRAPH);
    std::deque<Group> live;   // groups holding device memory, oldest first
    int next_job = 0;

    // Forms the next group and queues the uploads of its inputs on the
    // upload stream.
    auto prepare = [&](Group &g) {
        g.j0 = next_job;
        int64_t tri = 0;
        while (next_job < n && (next_job == g.j0 || tri + jobs[next_job].nt <= budget)) tri += jobs[next_job++].nt;
        g.j1 = next_job;
        const int gn = g.j1 - g.j0;
        g.dxy.assign(gn, nullptr);
        g.dtri.assign(gn, nullptr);
        g.up_rc = GP_OK;
        for (int k = 0; k < gn && g.up_rc == GP_OK; k++) {
            const gp_job &jb = jobs[g.j0 + k];
            g.up_rc = c->pool.alloc(8 * (size_t)std::max(jb.nv, 1), &g.dxy[k]);
            if (g.up_rc == GP_OK) g.up_rc = c->pool.alloc(12 * (size_t)std::max(jb.nt, 1), &g.dtri[k]);
            if (g.up_rc == GP_OK && jb.nv &&
                hipMemcpyAsync(g.dxy[k], jb.xy, 8 * (size_t)jb.nv, hipMemcpyHostToDevice, us) != hipSuccess)
                g.up_rc = GP_EHIP;
            if (g.up_rc == GP_OK && jb.nt &&
                hipMemcpyAsync(g.dtri[k], jb.tri, 12 * (size_t)jb.nt, hipMemcpyHostToDevice, us) != hipSuccess)
                g.up_rc = GP_EHIP;
        }
        if (g.up_rc == GP_OK && (hipEventCreateWithFlags(&g.uploaded, hipEventDisableTiming) != hipSuccess ||
                                 hipEventRecord(g.uploaded, us) != hipSuccess))
            g.up_rc = GP_EHIP;
        if (g.up_rc != GP_OK) (void)hipGetLastError();
    };

    Group cur;
    prepare(cur);
    while (true) {
        // 1. the next group's uploads, while this group builds
        Group nxt;
        const bool more = next_job < n;
        if (more) prepare(nxt);
        // 2. the previous group's downloads, overlapping both
        if (!live.empty() && !live.back().queued) group_download(jobs, live.back(), cs);
        // 3. this group's builds (after its uploads) and one meshing run
        const int gn = cur.j1 - cur.j0;
        if (cur.up_rc == GP_OK && hipStreamWaitEvent(s, cur.uploaded, 0) != hipSuccess) {
            (void)hipGetLastError();
            cur.up_rc = GP_EHIP;
        }
        if (cur.up_rc != GP_OK) {
            (void)hipStreamSynchronize(us);   // its uploads may still read the inputs
            for (int k = 0; k < gn; k++) jobs[cur.j0 + k].status = cur.up_rc;
        } else {
            std::vector<const int32_t *> pxy(gn), ptri(gn);
            std::vector<int32_t> nv(gn), nt(gn);
            std::vector<gp_mesh *> ms(gn, nullptr);
            std::vector<int> st(gn, GP_OK);
            for (int k = 0; k < gn; k++) {
                pxy[k] = static_cast<const int32_t *>(cur.dxy[k]);
                ptri[k] = static_cast<const int32_t *>(cur.dtri[k]);
                nv[k] = jobs[cur.j0 + k].nv;
                nt[k] = jobs[cur.j0 + k].nt;
            }
            const int b = gprt::build_many(c, gn, pxy.data(), nv.data(), ptri.data(), nt.data(), GP_IN_DEVICE,
                                           ms.data(), st.data());
            for (int k = 0; k < gn; k++) {
                const int r = b != GP_OK ? b : st[k];
                jobs[cur.j0 + k].status = r;
                if (r == GP_OK) {
                    cur.meshes.push_back(ms[k]);
                    cur.job.push_back(cur.j0 + k);
                }
            }
        }
        // the builds have drained the stream: the uploaded inputs are free
        for (void *p : cur.dxy) c->pool.release(p);
        for (void *p : cur.dtri) c->pool.release(p);
        cur.dxy.clear();
        cur.dtri.clear();
        if (!cur.meshes.empty()) {
            cur.res.assign(cur.meshes.size(), nullptr);
            const int mr =
                gpolylla_mesh_batch(c, cur.meshes.data(), (int32_t)cur.meshes.size(), mesh_flags, cur.res.data());
            if (mr != GP_OK) {
                for (int idx : cur.job) jobs[idx].status = mr;
                cur.res.clear();
                for (gp_mesh *m : cur.meshes) gpolylla_mesh_free(m);
                cur.meshes.clear();
                cur.job.clear();
            }
        }
        live.push_back(std::move(cur));
        // 4. at most two meshed groups hold memory: the one being downloaded
        //    and the one just queued
        while (live.size() > 2) {
            if (!live.front().queued) group_download(jobs, live.front(), cs);
            group_finish(live.front(), cs);
            live.pop_front();
        }
        if (!more) break;
        cur = std::move(nxt);
    }
    while (!live.empty()) {
        if (!live.front().queued) group_download(jobs, live.front(), cs);
        group_finish(live.front(), cs);
        live.pop_front();
    }
    (void)hipStreamDestroy(cs);
    (void)hipStreamDestroy(us);
    int rc_all = GP_OK;
    for (int i = 0; i < n; i++)
        if (jobs[i].status != GP_OK && rc_all == GP_OK) rc_all = jobs[i].status;
    return rc_all;
}

}  // extern "C"
