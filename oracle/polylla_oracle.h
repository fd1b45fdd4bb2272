/*
 * Sequential CPU oracle for the Polylla half-edge pipeline.
 *
 * TEST INFRASTRUCTURE ONLY.  This code defines the expected result that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * calls it, and it shares no code with the GPU library.
 *
 * It follows the sequential algorithm of the paper (Section 5, Algorithm 1:
 * label phase, traversal phase, repair phase) on the half-edge representation
 * of Section 4, with these fixed readings where the paper leaves a choice open:
 *   - coordinates are integers in [0, 2^30]; squared lengths and orientation
 *     tests are exact in int64;
 *   - triangles are stored counter-clockwise: a clockwise triple (a,b,c) is
 *     stored as (a,c,b); a zero-area triple is an error;
 *   - half-edge h = 3t+i starts at corner i of triangle t; next(h) = 3t+(i+1)%3,
 *     prev(h) = 3t+(i+2)%3; twin(h) = -1 on the boundary (no exterior
 *     half-edges);
 *   - edge order: the larger squared length wins; on equal squared length the
 *     lower edge id wins, where the edge id is min(h, twin(h)) (h when twin(h)
 *     is -1);
 *   - CW(h) = next(twin(h)), the next outgoing half-edge clockwise around
 *     origin(h);
 *   - barrier tips and their middle edges are found once, from the frontier
 *     labels of the label phase; the middle edge of a tip v whose single
 *     frontier edge leaves v as a is CW^k(a) with k = floor(degree(v)/2);
 *   - non-frontier half-edges get next = prev = -1;
 *   - output loops are listed by ascending minimum half-edge, each starting at
 *     that minimum.
 */
#ifndef POLYLLA_ORACLE_H
#define POLYLLA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_OK = 0,
    ORC_EINVAL = -1,       /* null pointer, negative count, index out of [0, nv) */
    ORC_ERANGE = -2,       /* coordinate outside [0, 2^30], or 3*nt >= 2^31 */
    ORC_EDEGEN = -3,       /* zero-area triangle */
    ORC_ENONMANIFOLD = -4, /* edge in > 2 triangles, or repeated directed edge */
    ORC_ENOMEM = -5,
    ORC_ECORRUPT = -10     /* a traversal did not close */
};

typedef struct {
    int64_t nt, nv, nh;
    int64_t nflipped;   /* triangles given clockwise and re-oriented */
    int64_t nties;      /* triangles whose largest squared length is shared */
    int64_t nterminal;  /* terminal edges, interior and boundary */
    int64_t ntips;      /* barrier tips */
    int64_t nmiddle;    /* distinct middle edges added by the repair */
    int64_t npoly;      /* output polygons */
    int64_t nloop_he;   /* half-edges on output loops */
    double ms_build, ms_label, ms_repair, ms_traverse, ms_canon;
} orc_stats;

/*
 * Runs the whole pipeline.  Inputs: xy[2*nv] (x0,y0,x1,y1,...), tri[3*nt].
 * Outputs (caller-allocated): org[3nt], twin[3nt], next_o[3nt], prev_o[3nt],
 * seeds[nt], loop_off[nt+1], loop_he[3nt].  Any output pointer except org and
 * twin may be NULL when not wanted.  Returns ORC_OK or a negative code.
 */
int orc_polylla(const int32_t *xy, int32_t nv, const int32_t *tri, int32_t nt,
                int32_t *org, int32_t *twin, int32_t *next_o, int32_t *prev_o,
                int32_t *seeds, int32_t *loop_off, int32_t *loop_he,
                uint8_t *longest_out, uint8_t *frontier_out, uint8_t *frontier_rep_out,
                orc_stats *st);

/* Builds only the half-edge structure (validation, orientation, twins). */
int orc_build(const int32_t *xy, int32_t nv, const int32_t *tri, int32_t nt,
              int32_t *org, int32_t *twin, orc_stats *st);

#ifdef __cplusplus
}
#endif
#endif
