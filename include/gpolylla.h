/*
 * gpolylla: Polylla polygonal meshing of 2-D triangulations on MI355X (gfx950).
 *
 * The problem statement follows the paper (Section 1 and Section 4.2): a
 * triangulation tau = (V, E) goes in as vertex coordinates and triangle index
 * triples; it is held as a half-edge structure on the device; the output is
 * the same half-edge structure with next/prev of the frontier half-edges
 * relinked so that each polygon of the Polylla mesh is one next-cycle, plus
 * one seed half-edge per polygon (Section 4.3: "output seed edges").
 *
 * Conventions (fixed where the paper leaves a choice open):
 *   - coordinates are int32 in [0, 2^30]; edge lengths are compared as exact
 *     int64 squared lengths; on equal squared length the edge with the lower
 *     id min(h, twin(h)) counts as longer;
 *   - each triangle is stored counter-clockwise (a clockwise triple (a,b,c)
 *     is stored as (a,c,b)); half-edge h = 3t+i starts at corner i of
 *     triangle t, next(h) = 3t+(i+1)%3, prev(h) = 3t+(i+2)%3; boundary
 *     half-edges have twin -1 (there are no exterior half-edges);
 *   - barrier tips (Section 3.1) are repaired in one pass from the
 *     label-phase frontier: for a tip v whose single frontier edge leaves v as
 *     a, the edge reached by floor(degree(v)/2) clockwise turns from a
 *     (CW(h) = next(twin(h))) becomes a frontier edge;
 *   - outputs: next[h], prev[h] = -1 for half-edges not on any polygon;
 *     seeds[p] ascending, each the minimum half-edge of its polygon's loop;
 *     loop_he[loop_off[p] .. loop_off[p+1]) is loop p starting at seeds[p]
 *     and following next.  All indices are local to their mesh.
 *
 * Return values: 0 (GP_OK) or a negative GP_E* code; gpolylla_strerror()
 * names it.  Functions never abort the process.
 *
 * Threading: a gp_ctx and everything built from it belong to one host thread
 * at a time.  A gp_server is safe to use from many threads.
 *
 * Lifetime: meshes and results hold memory of their context's pool; free them
 * before destroying the context.  Device memory released by a free is reused
 * only by later work on the same context stream, so frees never wait for the
 * GPU.
 */
#ifndef GPOLYLLA_H
#define GPOLYLLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define GP_OK 0
#define GP_EINVAL (-1)        /* null pointer, negative count, vertex index outside [0, nv) */
#define GP_ERANGE (-2)        /* coordinate outside [0, 2^30], or 3*nt >= 2^31 */
#define GP_EDEGEN (-3)        /* zero-area triangle */
#define GP_ENONMANIFOLD (-4)  /* an edge in more than two triangles, or a repeated directed edge */
#define GP_ENOMEM (-5)        /* device or pinned-host allocation failed, or the pool cap was hit */
#define GP_EHIP (-6)          /* a HIP runtime call failed */
#define GP_EAGAIN (-7)        /* server queue full */
#define GP_ETOOBIG (-8)       /* request footprint exceeds the server pool */
#define GP_ETIMEDOUT (-9)     /* wait timed out */
#define GP_ECORRUPT (-10)     /* a rotation, walk or scan guard tripped: the half-edge
                                 structure is not a valid manifold triangulation, or
                                 a turn around one vertex passed more than 2^20 edges
                                 (a vertex of that degree is beyond the supported range) */

/* ---- flags -------------------------------------------------------------- */
#define GP_IN_DEVICE 0x1u     /* build: xy and tri are device pointers on the context's device */
#define GP_COMPACT 0x8u       /* build: keep the mesh in the compact encoding (gpolylla_build_halfedges) */
#define GP_RENUMBER 0x40u     /* build: renumber along a Z-order curve first (gpolylla_build_halfedges) */
#define GP_ASYNC 0x2u         /* mesh: return once the work is queued; counts are read
                                 (and errors reported) by the first result query */
#define GP_GRAPH 0x4u         /* mesh: replay a captured hipGraph of the kernel chain; the
                                 graph is captured on the first call for a batch shape (the
                                 list of triangle counts) and reused while the shape repeats
                                 (up to 4 shapes per context; ignored when profiling, and
                                 for a single mesh small enough to run as one workgroup,
                                 which is one kernel launch either way) */
#define GP_OUT_LOOPS 0x10u    /* mesh: also produce seeds / loop_off / loop_he (default on) */
#define GP_OUT_NO_LOOPS 0x20u /* mesh: only next/prev and the counts */

typedef struct gp_ctx gp_ctx;
typedef struct gp_mesh gp_mesh;
typedef struct gp_result gp_result;
typedef struct gp_server gp_server;

typedef struct {
    size_t pool_bytes;  /* cap on device memory held by the context's pool; 0 = no cap */
    void *stream;       /* hipStream_t to run on; NULL = the context creates its own */
    int32_t profile;    /* 1 = record per-kernel HIP events (see gpolylla_ctx_kernel_ms) */
    int32_t block;      /* threads per block for the streaming kernels; 0 = tuned default */
    int32_t items;      /* items per thread for the streaming kernels; 0 = tuned default */
} gp_ctx_opts;

typedef struct {
    int64_t nt, nv, nh;   /* triangles, vertices, half-edges (3*nt) */
    int64_t npoly;        /* polygons (= seeds) */
    int64_t nloop_he;     /* half-edges on loops */
    int64_t nterminal;    /* terminal edges (interior and boundary) */
    int64_t ntips;        /* barrier tips repaired */
    int64_t nmiddle;      /* distinct middle edges added by the repair */
    int64_t nties;        /* triangles whose largest squared length is shared */
    int64_t nflipped;     /* triangles given clockwise (from the build) */
    int64_t loops_only;   /* 1: the result holds seeds and loops only (a server
                             started with loops_only): next'/prev' cannot be copied */
} gp_result_info;

typedef struct {      /* device views of a result (valid until gpolylla_result_free) */
    int32_t *next, *prev, *seeds, *loop_off, *loop_he;
} gp_result_dev;

/* ---- context ------------------------------------------------------------ */

/* Creates a context on HIP device `device`.  opts may be NULL. */
int gpolylla_ctx_create(int device, const gp_ctx_opts *opts, gp_ctx **out);
void gpolylla_ctx_destroy(gp_ctx *ctx);
/* Bytes currently held by the context's device pool (in use + cached). */
int gpolylla_ctx_pool_bytes(const gp_ctx *ctx, size_t *held, size_t *in_use);
/* With profile = 1: average device milliseconds per launch of each pipeline
 * kernel over the launches since the last reset.  names[i] receives a static
 * string.  Returns the number of kernels written (<= cap). */
int gpolylla_ctx_kernel_ms(gp_ctx *ctx, const char **names, double *avg_ms, int64_t *launches, int cap);
void gpolylla_ctx_kernel_reset(gp_ctx *ctx);

/* Launch shapes of the pipeline kernels (the autotuner's interface; no
 * passage of the paper fixes them).  spec is a comma-separated list of
 * "kernel=BxI" entries, any subset in any order:
 *   label=BxI, relink=BxI, compact=BxI   B threads per block (64..1024, a
 *                                        multiple of 64), I items per thread
 *                                        (1, 2, 4 or 8)
 *   persist=BxN                          the list-driven kernels: B threads
 *                                        per block, N blocks (1..65536)
 *   small=N                              batches whose meshes all have at
 *                                        most N triangles (0..4096; default
 *                                        4096) run as one workgroup per mesh
 *                                        with the whole pipeline in LDS, one
 *                                        launch, where the device's LDS per
 *                                        workgroup holds such a mesh (33
 *                                        bytes per triangle); 0: never
 * Tiles larger than a kernel's LDS staging allows (label 4096, relink 1024,
 * compact 2048 triangles) are reduced by halving I.  Results never depend on
 * the shapes.  Applies to runs started after the call; runs already queued
 * keep their shapes, and captured graphs are kept per shape.  Not to be
 * called concurrently with other calls on the same context.
 * Errors: GP_EINVAL for a null argument or any malformed entry, in which case
 * nothing changes. */
int gpolylla_ctx_set_launch(gp_ctx *ctx, const char *spec);
/* Writes the current shapes as a NUL-terminated spec of the form above into
 * buf (truncated to cap - 1 characters; buf may be NULL when cap is 0).
 * Returns the buffer size the whole spec needs (> 0), or GP_EINVAL. */
int gpolylla_ctx_get_launch(const gp_ctx *ctx, char *buf, int32_t cap);

/* ---- build -------------------------------------------------------------- */

/*
 * Builds the half-edge structure of a triangulation on the device
 * (Section 4.1-4.2): validation, counter-clockwise orientation (exact int64
 * orientation test) and twin matching (bucket half-edges by origin, then look
 * for the reverse edge in the target's bucket).
 *   xy:  2*nv int32, interleaved (x0, y0, x1, y1, ...)
 *   tri: 3*nt int32 vertex indices
 * Host pointers unless flags has GP_IN_DEVICE.  The inputs are copied; the
 * caller keeps ownership and may free them when the call returns.  On
 * success *out is a device-resident mesh owned by the caller (free it with
 * gpolylla_mesh_free).  Errors: GP_EINVAL, GP_ERANGE, GP_EDEGEN,
 * GP_ENONMANIFOLD, GP_ENOMEM, GP_EHIP.  Synchronous.
 * Numbering is kept as given, and the meshing kernels are fastest when it is
 * spatially coherent (grid rows, a space-filling curve): neighbours then
 * share cache lines and tiles.  A randomly numbered 33.5M-triangle grid
 * meshes about 9x slower than the same grid numbered by rows; results are
 * the same either way, up to ties, which the numbering breaks.
 * GP_COMPACT keeps the mesh in a narrower encoding, for bigger meshes per
 * device (the direction Section 8 names for future work): per triangle its
 * first corner (int32) and the other two as 16-bit offsets from it, per
 * half-edge its twin as a 16-bit offset from itself, and the few values
 * whose offsets do not fit in a hash table.  About 14 bytes per triangle
 * instead of 24 (xy unchanged); every meshing call gives the same results
 * as with the int32 arrays.
 * GP_RENUMBER first renumbers the input on the device, vertices in the
 * Z-order (Morton) order of their coordinates and triangles in that of their
 * centroids (corners keep their order within a triangle), which restores the
 * locality the kernels need to input numbered without it.  The mesh, and
 * every result of meshing it, are then in the new numbering, exactly as if
 * the caller had passed the renumbered input; gpolylla_mesh_permutation
 * gives the maps back to the caller's numbering.  Ties between equal edge
 * lengths are broken by edge id (Section 2 reading), so they may fall
 * differently than in the original numbering.
 */
int gpolylla_build_halfedges(gp_ctx *ctx, const int32_t *xy, int32_t nv, const int32_t *tri,
                             int32_t nt, uint32_t flags, gp_mesh **out);
/* Copies the oriented corner list (org, 3*nt) and twins (3*nt) to host buffers
 * (decoded, for a compact mesh); either may be NULL.  nflipped (may be NULL)
 * receives the re-oriented count. */
int gpolylla_mesh_copy(const gp_mesh *mesh, int32_t *org, int32_t *twin, int64_t *nflipped);
int gpolylla_mesh_size(const gp_mesh *mesh, int32_t *nv, int32_t *nt);
/* The maps of a renumbered mesh (GP_RENUMBER) back to the caller's
 * numbering: tri_new_to_old (nt) and vert_new_to_old (nv), host buffers,
 * either may be NULL.  GP_EINVAL for a mesh built without GP_RENUMBER. */
int gpolylla_mesh_permutation(const gp_mesh *mesh, int32_t *tri_new_to_old, int32_t *vert_new_to_old);
/* Device bytes the mesh holds (coordinates, corners, twins; in a compact
 * mesh the escape table too); escapes (may be NULL) receives the number of
 * escaped values of a compact mesh (0 otherwise). */
int gpolylla_mesh_bytes(const gp_mesh *mesh, size_t *bytes, int64_t *escapes);
void gpolylla_mesh_free(gp_mesh *mesh);

/* ---- meshing ------------------------------------------------------------ */

/*
 * Runs the Polylla pipeline on one resident mesh: longest-edge, frontier and
 * seed labelling (Section 6.1-6.3), relinking next/prev of frontier
 * half-edges (Section 6.5), barrier-tip repair (Section 6.4, one pass), seed
 * walks to each loop's minimum (Sections 6.5.1-6.6) and compaction of the
 * seeds and loops (Section 6.7).  The mesh is not modified.  On success *out
 * holds device-resident results owned by the caller.  Errors: GP_EINVAL,
 * GP_ENOMEM, GP_EHIP, GP_ECORRUPT.  Synchronous unless GP_ASYNC.
 */
int gpolylla_mesh(gp_ctx *ctx, const gp_mesh *mesh, uint32_t out_flags, gp_result **out);

/*
 * Runs n meshes as one batch: every kernel of the pipeline is launched once
 * for all meshes over a flattened tile space with a per-mesh descriptor
 * table, so uneven sizes share launches.  Results are identical to n calls
 * of gpolylla_mesh; out[i] belongs to meshes[i].  Meshes may repeat.
 */
int gpolylla_mesh_batch(gp_ctx *ctx, const gp_mesh *const *meshes, int32_t n, uint32_t out_flags,
                        gp_result **out);

/* Counts of a result (waits for an asynchronous run). */
int gpolylla_result_info(gp_result *res, gp_result_info *info);
/* Copies outputs to caller-allocated host buffers sized from the info
 * (next, prev: nh; seeds: npoly; loop_off: npoly+1; loop_he: nloop_he).
 * NULL skips an output.  GP_EINVAL when next or prev is asked of a result
 * that holds loops only (info.loops_only). */
int gpolylla_result_copy(gp_result *res, int32_t *next, int32_t *prev, int32_t *seeds,
                         int32_t *loop_off, int32_t *loop_he);
/* Device pointers of the outputs, for zero-copy consumers. */
int gpolylla_result_device(gp_result *res, gp_result_dev *dev);
void gpolylla_result_free(gp_result *res);

/* Waits until all queued work of the context has finished. */
int gpolylla_ctx_sync(gp_ctx *ctx);

/* ---- intermediate stages (debugging) ------------------------------------- */

/*
 * With debug on (gpolylla_ctx_set_debug), every meshing run of the context
 * keeps copies of its intermediate stages, so that a mismatch can be traced
 * to the step that made it: the label bytes and next'/prev' as the relink
 * left them (Sections 6.1-6.3 and 6.5: before the repair of Section 6.4),
 * the barrier tips the relink found (half-edges h with next'(h) == twin(h)),
 * and the label bytes at the end.  Label byte of triangle t: bits 0-1 the
 * local index of its longest edge, bits 2-4 the frontier bits of its edges
 * 0-2, bit 5 set when its longest edge is a terminal edge whose seed is in t.
 * Debug runs do not use captured graphs and cost the copies.
 */
int gpolylla_ctx_set_debug(gp_ctx *ctx, int32_t on);

/* Host buffers (each may be NULL) for gpolylla_result_debug. */
typedef struct {
    uint8_t *tflag_relink;   /* nt */
    int32_t *next_relink;    /* 3*nt */
    int32_t *prev_relink;    /* 3*nt */
    uint8_t *tflag_final;    /* nt */
    int32_t *tips;           /* tips_cap: the mesh's barrier tips, in no particular order */
    int32_t tips_cap;
    int32_t ntips;           /* out: the mesh's tip count (may exceed tips_cap) */
} gp_result_debug;

/* Copies a debug run's intermediate stages of one result (waits for the run).
 * GP_EINVAL when the result did not come from a debug run; the run's own
 * status otherwise (GP_ECORRUPT still copies, for inspection). */
int gpolylla_result_debug(gp_result *res, gp_result_debug *out);

/* ---- host-to-host jobs with overlapped copies ---------------------------- */

/*
 * The paper measures the copies to and from the device beside the kernels
 * (Section 7, the copy columns of Table 1) and finds that they take most of
 * the time of a run (Section 8).  gpolylla_mesh_jobs takes triangulations in
 * host memory and returns their polygons in host memory, overlapping the
 * copies of one group of jobs with the copies, builds and meshing of the
 * next: in a long enough list the time per job approaches that of its slower
 * copy direction, not the sum of all steps.
 *
 * One job: inputs as for gpolylla_build_halfedges (host xy: 2*nv int32, tri:
 * 3*nt int32); outputs into caller-allocated host buffers of capacity
 * next, prev: 3*nt (both NULL: only the loops are copied back);
 * seeds: nt; loop_off: nt + 1; loop_he: 3*nt.  npoly and nloop_he receive
 * the counts (the filled lengths are npoly, npoly + 1 and nloop_he), status
 * the job's own result (a build error, GP_ECORRUPT, ...).  The buffers must
 * stay valid until the call returns; pinned host memory (hipHostMalloc) is
 * needed for the copies to overlap (pageable memory works, serialised).
 */
typedef struct {
    const int32_t *xy;
    int32_t nv;
    const int32_t *tri;
    int32_t nt;
    int32_t *next, *prev;
    int32_t *seeds, *loop_off, *loop_he;
    int32_t npoly, nloop_he;   /* out */
    int32_t status;            /* out */
    int32_t reserved;
} gp_job;

/*
 * Meshes jobs[0..n) in order.  Consecutive jobs are grouped up to
 * group_triangles triangles (0: 8M; a larger job is a group of its own) and
 * each group is one batched run (gpolylla_mesh_batch); flags: 0 or GP_GRAPH.
 * A list whose jobs all have at most 4096 triangles and 4096 vertices (and
 * fit the device's LDS per workgroup) runs packed instead: per group one
 * upload of every job's inputs from a pinned staging block, one launch that
 * builds and meshes each job in a workgroup of its own (the same checks and
 * error codes as gpolylla_build_halfedges), and one download; flags are
 * then ignored.
 * Uses the context's stream for uploads, builds and runs, and a stream of its
 * own for the downloads; returns when every job's outputs are in host memory.
 * Returns GP_OK when every job succeeded, else the first failed job's status
 * (every job's own status is set either way); GP_EINVAL for a null or
 * inconsistent argument (nothing run).  Not to be called concurrently with
 * other calls on the same context.
 */
int gpolylla_mesh_jobs(gp_ctx *ctx, gp_job *jobs, int32_t n, int64_t group_triangles, uint32_t flags);

/* ---- meshing without allocation ----------------------------------------- */

/* Counts of one gpolylla_mesh_noalloc run, written by the device when the run
 * completes (the same counts gpolylla_result_info reports). */
typedef struct {
    int32_t status;       /* GP_OK, or GP_ECORRUPT when a device guard tripped */
    int32_t npoly;        /* polygons (= seeds) */
    int32_t nloop_he;     /* half-edges on loops */
    int32_t ntips;        /* barrier tips repaired */
    int32_t nmiddle;      /* distinct middle edges added by the repair */
    int32_t nties;        /* triangles whose largest squared length is shared */
    int32_t reserved[2];  /* written as 0 */
} gp_dev_counts;

/* Size of the library's per-device scratch array for gpolylla_mesh_noalloc. */
#define GP_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/*
 * For callers that cannot allocate: code under HIP graph capture, serving
 * loops and harnesses that forbid hipMalloc.  The same meshing run as
 * gpolylla_mesh (the same kernels, results identical element by element), with
 * no device, pinned-host or pool allocation and no host synchronisation: it
 * returns once the run is queued on the context's stream.
 *   mesh:   built beforehand by gpolylla_build_halfedges on this context
 *   out:    caller-allocated device buffers on the context's device, at least
 *           next, prev: 3*nt + 1 int32; seeds: nt + 1; loop_off: nt + 2;
 *           loop_he: 3*nt + 1 (the entries past the counts are scratch)
 *   counts: caller-allocated device memory; receives the counts of the run
 * The run's scratch (labels, lists, per-tile totals) lives in one static
 * array of GP_NOALLOC_SCRATCH_BYTES per device, set up by gpolylla_ctx_create
 * and held until the process ends; a mesh whose scratch does not fit (above
 * about 4.0 million triangles with the default launch shapes) is refused with
 * GP_ETOOBIG before anything is queued.  Every call on one device shares
 * that array: calls on one context are ordered by its stream, and calls that
 * overlap on one device (other contexts or streams) race and must not be made.
 * Errors: GP_EINVAL (null argument, mesh of another context), GP_ETOOBIG,
 * GP_EHIP (the scratch array could not be located at set-up, or a launch
 * failed).  Errors found by the kernels arrive in counts->status.
 */
int gpolylla_mesh_noalloc(gp_ctx *ctx, const gp_mesh *mesh, const gp_result_dev *out, gp_dev_counts *counts);

/* ---- serving ------------------------------------------------------------ */

typedef struct {
    size_t pool_bytes;   /* device bytes for requests in flight, split over the lanes; 0 = 16 GiB */
    int32_t max_batch;   /* requests per batched run; 0 = 64 */
    int32_t max_queue;   /* queued requests before GP_EAGAIN; 0 = 4096 */
    int32_t n_lanes;     /* streams whose batches overlap on the device (1..8); 0 = 2 */
    int32_t loops_only;  /* 1: results hold seeds and loops only, not next'/prev' (a
                            polygon is given by its loop; the download shrinks to a third) */
} gp_serve_opts;

typedef struct {
    int64_t submitted, completed, rejected, failed, batches, in_flight;
    double p50_ms, p99_ms, mean_ms, max_ms;   /* arrival (or submit) -> result on the host */
    double mtri_s;                            /* triangles completed per second, first submit to last result */
} gp_serve_stats;

/*
 * Starts a server on the device of ctx (whose launch shapes it copies).  The
 * server owns its own streams, threads and device memory: n_lanes lanes,
 * each with a stream, a host thread and an arena of pool_bytes / n_lanes
 * bytes.  Submitted inputs are copied into pinned host buffers that the
 * server reuses after requests complete (at most 4 GiB of them kept free).  A request is admitted into a batch when the
 * exact device footprint of the batch (every half-edge build plus the
 * batched meshing run) fits a lane's arena.  Batches on different lanes
 * overlap; requests that arrive while batches run join the next free lane
 * (continuous batching).  With loops_only, only the seeds and loops of each
 * result are copied back (next'/prev' stay on the device and are dropped).
 * ctx itself is not used after the call.
 */
int gpolylla_serve_start(gp_ctx *ctx, const gp_serve_opts *opts, gp_server **out);
/* Queues a triangulation (host arrays, copied before return).  Errors:
 * GP_EINVAL, GP_ERANGE, GP_ETOOBIG (footprint above one lane's arena),
 * GP_EAGAIN (queue full).  Thread-safe. */
int gpolylla_serve_submit(gp_server *srv, const int32_t *xy, int32_t nv, const int32_t *tri, int32_t nt,
                          uint64_t *ticket);
/* The same, for a request that arrived at arrival_ns (CLOCK_MONOTONIC
 * nanoseconds, the clock of std::chrono::steady_clock and of Python's
 * time.monotonic_ns): its latency runs from then, so time the caller spent
 * before submitting (its own queueing, the copy of the inputs) is counted.
 * arrival_ns <= 0: now.  GP_EINVAL for an arrival in the future. */
int gpolylla_serve_submit_at(gp_server *srv, const int32_t *xy, int32_t nv, const int32_t *tri, int32_t nt,
                             int64_t arrival_ns, uint64_t *ticket);
/* Waits for a ticket (timeout_ms < 0: forever).  On success *out is a
 * host-resident result (gpolylla_result_info / _copy / _free work on it;
 * gpolylla_result_device does not).  Returns the request's status (its build
 * or meshing error), GP_ETIMEDOUT, or GP_EINVAL for an unknown ticket.  A
 * ticket can be waited for once; while one thread waits for it, a wait from
 * another thread returns GP_EINVAL at once (after GP_ETIMEDOUT it can be
 * waited for again).  Thread-safe. */
int gpolylla_serve_wait(gp_server *srv, uint64_t ticket, int32_t timeout_ms, gp_result **out);
int gpolylla_serve_stats(gp_server *srv, gp_serve_stats *stats);
/* Clears the latency and throughput statistics (after a warm-up).  Requests
 * not finished yet count as submitted afterwards. */
int gpolylla_serve_reset_stats(gp_server *srv);
/* Finishes every queued request, then stops.  Results already handed out
 * stay valid until freed. */
int gpolylla_serve_stop(gp_server *srv);

const char *gpolylla_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
