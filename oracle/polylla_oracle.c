/*
 * Sequential CPU oracle for the Polylla half-edge pipeline.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the GPU library.  Conventions are listed in polylla_oracle.h.
 *
 * Phases, in the paper's order (Section 5, Algorithm 1):
 *   build     validate, orient, half-edges; twins by sorting undirected edge
 *             keys (Section 4.1-4.2 describe the structure; building it is
 *             host work there too)
 *   label     Algorithm 2 (longest edge per triangle), Algorithm 3 (frontier
 *             edges), Algorithm 4 (seed edges on terminal edges)
 *   repair    the labelling half of Algorithm 6: barrier tips (Section 3.1:
 *             an endpoint touching exactly one frontier edge) get their middle
 *             edge added to the frontier and both of its half-edges become
 *             seeds; tips are taken from the label-phase frontier in one pass
 *   traverse  Algorithm 5 from every seed over the final frontier, skipping
 *             seeds whose polygon already exists (the usage check of
 *             Algorithm 6)
 *   canon     loops listed by ascending minimum half-edge
 */
#define _POSIX_C_SOURCE 199309L
#include "polylla_oracle.h"

#include <stdlib.h>
#include <string.h>
#include <time.h>

#define COORD_MAX (1 << 30)

static double now_ms(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec * 1e3 + ts.tv_nsec * 1e-6;
}

/* ---- half-edge queries of Section 4.1, implicit triangle layout ---------- */

static inline int64_t he_next(int64_t h) { return (h % 3 == 2) ? h - 2 : h + 1; }
static inline int64_t he_prev(int64_t h) { return (h % 3 == 0) ? h + 2 : h - 1; }

/* squared length of the edge origin(h) -> target(h) */
static int64_t sq_len(const int32_t *xy, const int32_t *org, int64_t h) {
    int64_t a = org[h], b = org[he_next(h)];
    int64_t dx = (int64_t)xy[2 * b] - xy[2 * a];
    int64_t dy = (int64_t)xy[2 * b + 1] - xy[2 * a + 1];
    return dx * dx + dy * dy;
}

/* ---- build ---------------------------------------------------------------- */

typedef struct {
    int32_t lo, hi; /* undirected key */
    int32_t h;      /* half-edge */
} edge_rec;

static int cmp_edge(const void *pa, const void *pb) {
    const edge_rec *a = (const edge_rec *)pa, *b = (const edge_rec *)pb;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
    return (a->h > b->h) - (a->h < b->h);
}

int orc_build(const int32_t *xy, int32_t nv, const int32_t *tri, int32_t nt,
              int32_t *org, int32_t *twin, orc_stats *st) {
    if (nv < 0 || nt < 0) return ORC_EINVAL;
    if ((nv > 0 && !xy) || (nt > 0 && (!tri || !org || !twin))) return ORC_EINVAL;
    if (3 * (int64_t)nt >= ((int64_t)1 << 31)) return ORC_ERANGE;
    int64_t nh = 3 * (int64_t)nt;
    for (int64_t v = 0; v < nv; v++) {
        if (xy[2 * v] < 0 || xy[2 * v] > COORD_MAX || xy[2 * v + 1] < 0 || xy[2 * v + 1] > COORD_MAX)
            return ORC_ERANGE;
    }
    int64_t flipped = 0;
    for (int64_t t = 0; t < nt; t++) {
        int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
        if (a < 0 || a >= nv || b < 0 || b >= nv || c < 0 || c >= nv) return ORC_EINVAL;
        int64_t abx = (int64_t)xy[2 * b] - xy[2 * a], aby = (int64_t)xy[2 * b + 1] - xy[2 * a + 1];
        int64_t acx = (int64_t)xy[2 * c] - xy[2 * a], acy = (int64_t)xy[2 * c + 1] - xy[2 * a + 1];
        int64_t o = abx * acy - aby * acx; /* twice the signed area */
        if (o == 0) return ORC_EDEGEN;
        if (o < 0) { int32_t s = b; b = c; c = s; flipped++; }
        org[3 * t] = a;
        org[3 * t + 1] = b;
        org[3 * t + 2] = c;
    }
    /* Twins: sort the undirected keys; an edge seen once is boundary, an edge
     * seen twice must appear once in each direction. */
    edge_rec *rec = (edge_rec *)malloc(sizeof(edge_rec) * (size_t)(nh ? nh : 1));
    if (!rec) return ORC_ENOMEM;
    for (int64_t h = 0; h < nh; h++) {
        int32_t u = org[h], v = org[he_next(h)];
        rec[h].lo = u < v ? u : v;
        rec[h].hi = u < v ? v : u;
        rec[h].h = (int32_t)h;
    }
    qsort(rec, (size_t)nh, sizeof(edge_rec), cmp_edge);
    int rc = ORC_OK;
    for (int64_t i = 0; i < nh;) {
        int64_t j = i + 1;
        while (j < nh && rec[j].lo == rec[i].lo && rec[j].hi == rec[i].hi) j++;
        if (j - i == 1) {
            twin[rec[i].h] = -1;
        } else if (j - i == 2) {
            int32_t h1 = rec[i].h, h2 = rec[i + 1].h;
            if (org[h1] == org[h2]) { rc = ORC_ENONMANIFOLD; break; }
            twin[h1] = h2;
            twin[h2] = h1;
        } else {
            rc = ORC_ENONMANIFOLD;
            break;
        }
        i = j;
    }
    free(rec);
    if (st) {
        st->nt = nt;
        st->nv = nv;
        st->nh = nh;
        st->nflipped = flipped;
    }
    return rc;
}

/* ---- label phase ------------------------------------------------------------ */

/* edge id of Convention "lower edge id wins" */
static inline int64_t edge_id(const int32_t *twin, int64_t h) {
    return (twin[h] >= 0 && twin[h] < h) ? twin[h] : h;
}

/* 1 when edge a precedes edge b as the longer one */
static inline int longer(int64_t la, int64_t ida, int64_t lb, int64_t idb) {
    return la > lb || (la == lb && ida < idb);
}

/* ---- pipeline ------------------------------------------------------------- */

int orc_polylla(const int32_t *xy, int32_t nv, const int32_t *tri, int32_t nt,
                int32_t *org, int32_t *twin, int32_t *next_o, int32_t *prev_o,
                int32_t *seeds, int32_t *loop_off, int32_t *loop_he,
                uint8_t *longest_out, uint8_t *frontier_out, uint8_t *frontier_rep_out,
                orc_stats *st) {
    orc_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    double t0 = now_ms();
    int rc = orc_build(xy, nv, tri, nt, org, twin, st);
    if (rc != ORC_OK) return rc;
    double t1 = now_ms();
    st->ms_build = t1 - t0;
    int64_t nh = 3 * (int64_t)nt;
    size_t nb = (size_t)(nh ? nh : 1);

    uint8_t *longest = (uint8_t *)calloc(nb, 1);   /* longest-edge bitvector */
    uint8_t *front = (uint8_t *)calloc(nb, 1);     /* frontier-edge bitvector */
    uint8_t *front2 = (uint8_t *)calloc(nb, 1);    /* frontier after repair */
    uint8_t *visited = (uint8_t *)calloc(nb, 1);   /* usage: already on a loop */
    uint8_t *middle = (uint8_t *)calloc(nb, 1);    /* half-edge of a middle edge */
    /* seed-list, followed by the subseed-list (two entries per tip) */
    int32_t *seedl = (int32_t *)malloc(sizeof(int32_t) * (nb + 2 * (size_t)(nv > 0 ? nv : 0)));
    int32_t *nx = (int32_t *)malloc(sizeof(int32_t) * nb);
    int32_t *pv = (int32_t *)malloc(sizeof(int32_t) * nb);
    int32_t *fcount = (int32_t *)calloc((size_t)(nv ? nv : 1), sizeof(int32_t));
    int32_t *vhe = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv ? nv : 1));
    if (!longest || !front || !front2 || !visited || !middle || !seedl || !nx || !pv || !fcount || !vhe) {
        rc = ORC_ENOMEM;
        goto done;
    }

    /* Algorithm 2: longest edge of each triangle. */
    for (int64_t t = 0; t < nt; t++) {
        int64_t best = 3 * t, bl = sq_len(xy, org, best), bid = edge_id(twin, best);
        for (int i = 1; i < 3; i++) {
            int64_t h = 3 * t + i, l = sq_len(xy, org, h), id = edge_id(twin, h);
            if (longer(l, id, bl, bid)) { best = h; bl = l; bid = id; }
        }
        int n_at_max = 0;
        for (int i = 0; i < 3; i++) n_at_max += sq_len(xy, org, 3 * t + i) == bl;
        int ties = n_at_max > 1;
        st->nties += ties;
        longest[best] = 1;
    }
    /* Algorithm 3: frontier edges, i.e. boundary edges and edges that are the
     * longest edge of neither adjacent triangle (Definition 3 and Section 5.1). */
    for (int64_t h = 0; h < nh; h++) {
        int32_t g = twin[h];
        front[h] = (g < 0) || (!longest[h] && !longest[g]);
    }
    /* Algorithm 4: one seed per terminal edge (interior: longest on both
     * sides, the lower half-edge is the seed; boundary: longest of its only
     * triangle). */
    int64_t nseed = 0;
    for (int64_t h = 0; h < nh; h++) {
        int32_t g = twin[h];
        if (longest[h] && (g < 0 || (longest[g] && h < g))) seedl[nseed++] = (int32_t)h;
    }
    st->nterminal = nseed;
    double t2 = now_ms();
    st->ms_label = t2 - t1;

    /* Repair labelling (first half of Algorithm 6), from the label-phase
     * frontier.  Frontier edges are counted per edge at both endpoints. */
    for (int64_t h = 0; h < nh; h++) {
        int32_t g = twin[h];
        if (front[h] && (g < 0 || h < g)) {
            fcount[org[h]]++;
            fcount[org[he_next(h)]]++;
        }
    }
    for (int64_t v = 0; v < nv; v++) vhe[v] = -1;
    for (int64_t h = nh - 1; h >= 0; h--) vhe[org[h]] = (int32_t)h;
    memcpy(front2, front, nb);
    int64_t nsub = 0;
    int32_t *subseed = seedl + nseed; /* subseed-list follows the seed-list */
    for (int64_t v = 0; v < nv; v++) {
        if (fcount[v] != 1) continue;
        st->ntips++;
        /* edgeOfVertex, then clockwise until the frontier edge */
        int64_t e = vhe[v], guard = 0;
        while (!front[e]) {
            if (twin[e] < 0 || ++guard > nh) { rc = ORC_ECORRUPT; goto done; }
            e = he_next(twin[e]);
        }
        /* degree: outgoing half-edges met on a full clockwise turn */
        int64_t d = 0, r = e;
        do {
            if (twin[r] < 0 || ++d > nh) { rc = ORC_ECORRUPT; goto done; }
            r = he_next(twin[r]);
        } while (r != e);
        int64_t m = e;
        for (int64_t k = 0; k < d / 2; k++) m = he_next(twin[m]);
        int32_t mt = twin[m];
        if (!middle[m]) st->nmiddle++;
        middle[m] = middle[mt] = 1;
        front2[m] = front2[mt] = 1;
        subseed[nsub++] = (int32_t)m;
        subseed[nsub++] = mt;
    }
    double t3 = now_ms();
    st->ms_repair = t3 - t2;

    /* Algorithm 5 from each seed over the final frontier. */
    for (int64_t h = 0; h < nh; h++) nx[h] = pv[h] = -1;
    for (int64_t s = 0; s < nseed + nsub; s++) {
        int64_t he = seedl[s], guard = 0;
        while (!front2[he]) {  /* move to a frontier edge around origin(he) */
            if (twin[he] < 0 || ++guard > nh) { rc = ORC_ECORRUPT; goto done; }
            he = he_next(twin[he]);
        }
        if (visited[he]) continue; /* this polygon was generated already */
        int64_t init = he, out_curr = init, steps = 0;
        do {
            int64_t in_curr = he_next(out_curr), rot = 0;
            while (!front2[in_curr]) { /* clockwise around target(out_curr) */
                if (twin[in_curr] < 0 || ++rot > nh) { rc = ORC_ECORRUPT; goto done; }
                in_curr = he_next(twin[in_curr]);
            }
            nx[out_curr] = (int32_t)in_curr;
            pv[in_curr] = (int32_t)out_curr;
            visited[out_curr] = 1;
            out_curr = in_curr;
            if (++steps > nh) { rc = ORC_ECORRUPT; goto done; }
        } while (out_curr != init);
    }
    double t4 = now_ms();
    st->ms_traverse = t4 - t3;

    /* Canonical order: scanning half-edges upward, the first unlisted
     * frontier half-edge is the minimum of its loop. */
    {
        int64_t p = 0, f = 0;
        memset(visited, 0, nb);
        for (int64_t h = 0; h < nh; h++) {
            if (!front2[h] || visited[h]) continue;
            if (seeds) seeds[p] = (int32_t)h;
            if (loop_off) loop_off[p] = (int32_t)f;
            int64_t c = h;
            do {
                if (c < 0 || visited[c]) { rc = ORC_ECORRUPT; goto done; }
                visited[c] = 1;
                if (loop_he) loop_he[f] = (int32_t)c;
                f++;
                c = nx[c];
            } while (c != h);
            p++;
        }
        if (loop_off) loop_off[p] = (int32_t)f;
        st->npoly = p;
        st->nloop_he = f;
    }
    st->ms_canon = now_ms() - t4;
    if (next_o) memcpy(next_o, nx, sizeof(int32_t) * (size_t)nh);
    if (prev_o) memcpy(prev_o, pv, sizeof(int32_t) * (size_t)nh);
    if (longest_out) memcpy(longest_out, longest, (size_t)nh);
    if (frontier_out) memcpy(frontier_out, front, (size_t)nh);
    if (frontier_rep_out) memcpy(frontier_rep_out, front2, (size_t)nh);

done:
    free(longest); free(front); free(front2); free(visited); free(middle);
    free(seedl); free(nx); free(pv); free(fcount); free(vhe);
    return rc;
}
