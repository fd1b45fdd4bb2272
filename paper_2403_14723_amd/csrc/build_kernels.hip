// Half-edge construction on the device (the structure of Section 4.1-4.2,
// built on the GPU instead of the host).
//
//   k_check_xy   coordinates in [0, 2^30]
//   k_orient     index check, exact int64 orientation test, counter-clockwise
//                corner order, out-degree count per vertex
//   k_scan_excl  exclusive scan of the out-degrees (decoupled look-back)
//   k_bucket     half-edges grouped by origin vertex (CSR), each with its
//                target vertex beside it
//   k_match      twin(h) for h = u->v: the half-edge v->u in v's bucket; two
//                v->u, or (for an h with none) a second u->v in u's
//                bucket, is non-manifold
//
// Errors are reduced with a 64-bit atomicMin over (rank << 8 | code) so the
// reported code is deterministic: coordinate range first, then the lowest
// bad triangle, then the lowest non-manifold half-edge.
#include "gp_internal.h"

namespace gp {

namespace {

constexpr int kCoordMax = 1 << 30;
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr uint64_t kScanAgg = 1ull << 62;
constexpr uint64_t kScanInc = 2ull << 62;
// k_orient and k_bucket work in tiles of 256 threads x kTileItems items and
// count per vertex in an LDS histogram when the tile's vertex ids span at
// most kHistBins (meshes numbered row by row or along a curve do): one
// global atomic per distinct vertex of the tile instead of one per corner
constexpr int kTileItems = 4;
constexpr int kHistBins = 8192;

// [lo, hi] of the values v over the block (hi < lo when no thread has one);
// every thread calls it, s_lohi is shared
__device__ __forceinline__ void block_range(int vlo, int vhi, int *s_lohi, int &lo, int &hi) {
    if (threadIdx.x == 0) {
        s_lohi[0] = 0x7fffffff;
        s_lohi[1] = -1;
    }
    __syncthreads();
    if (vhi >= vlo) {
        atomicMin(&s_lohi[0], vlo);
        atomicMax(&s_lohi[1], vhi);
    }
    __syncthreads();
    lo = s_lohi[0];
    hi = s_lohi[1];
}

__device__ __forceinline__ unsigned long long err_key(unsigned long long rank, int code) {
    return (rank << 8) | (unsigned long long)(-code);
}

__device__ __forceinline__ int he_next_b(int h) {
    int t = h / 3;
    return (h - 3 * t == 2) ? h - 2 : h + 1;
}

__global__ void k_check_xy(const int2 *__restrict__ xy, int nv, unsigned long long *err) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
        int2 p = xy[v];
        if (p.x < 0 || p.x > kCoordMax || p.y < 0 || p.y > kCoordMax) atomicMin(err, err_key(0, -2));
    }
}

__global__ void __launch_bounds__(256) k_orient(const int2 *__restrict__ xy, const int32_t *__restrict__ tri,
                                                 int nv, int nt, int32_t *__restrict__ org,
                                                 int32_t *__restrict__ deg, unsigned long long *err,
                                                 int32_t *nflipped) {
    __shared__ int s_hist[kHistBins];
    __shared__ int s_lohi[2];
    const int TB = 256 * kTileItems;
    for (int base = blockIdx.x * TB; base < nt; base += gridDim.x * TB) {   // block-uniform
        int cv[kTileItems][3];
        bool ok[kTileItems];
        int vlo = 0x7fffffff, vhi = -1, nflip = 0;
#pragma unroll
        for (int j = 0; j < kTileItems; j++) {
            const int t = base + j * 256 + threadIdx.x;
            ok[j] = false;
            bool flip = false;
            if (t < nt) {
                int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
                if ((unsigned)a >= (unsigned)nv || (unsigned)b >= (unsigned)nv || (unsigned)c >= (unsigned)nv) {
                    atomicMin(err, err_key(1ull + t, -1));
                } else {
                    int2 pa = xy[a], pb = xy[b], pc = xy[c];
                    long long o = ((long long)pb.x - pa.x) * ((long long)pc.y - pa.y) -
                                  ((long long)pb.y - pa.y) * ((long long)pc.x - pa.x);
                    if (o == 0) {
                        atomicMin(err, err_key(1ull + t, -3));
                    } else {
                        if (o < 0) {
                            int s = b;
                            b = c;
                            c = s;
                            flip = true;
                        }
                        org[3 * t] = a;
                        org[3 * t + 1] = b;
                        org[3 * t + 2] = c;
                        cv[j][0] = a;
                        cv[j][1] = b;
                        cv[j][2] = c;
                        ok[j] = true;
                        vlo = min(vlo, min(a, min(b, c)));
                        vhi = max(vhi, max(a, max(b, c)));
                    }
                }
            }
            const unsigned long long m = __ballot(flip);
            nflip += __popcll(m);
        }
        if (nflip && __lane_id() == 0) atomicAdd(nflipped, nflip);
        int lo, hi;
        block_range(vlo, vhi, s_lohi, lo, hi);
        if (hi >= lo && hi - lo < kHistBins) {   // block-uniform
            const int range = hi - lo + 1;
            for (int k = threadIdx.x; k < range; k += 256) s_hist[k] = 0;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kTileItems; j++)
                if (ok[j])
#pragma unroll
                    for (int i = 0; i < 3; i++) atomicAdd(&s_hist[cv[j][i] - lo], 1);
            __syncthreads();
            for (int k = threadIdx.x; k < range; k += 256) {
                const int n = s_hist[k];
                if (n) atomicAdd(&deg[lo + k], n);
            }
        } else {
#pragma unroll
            for (int j = 0; j < kTileItems; j++)
                if (ok[j])
#pragma unroll
                    for (int i = 0; i < 3; i++) atomicAdd(&deg[cv[j][i]], 1);
        }
        __syncthreads();   // the histogram and range are reused by the next tile
    }
}

// Exclusive scan of in[0, n) into out[0, n], out[n] = total.  One pass with
// dynamically numbered tiles and decoupled look-back.
__global__ void __launch_bounds__(kScanBlock) k_scan_excl(const int32_t *__restrict__ in, int32_t *out,
                                                           int n, uint64_t *status, int32_t *tile_ctr,
                                                           unsigned long long *err) {
    __shared__ int s_tile;
    __shared__ int s_wave[kScanBlock / 64];
    __shared__ int s_prefix;
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1);
    __syncthreads();
    const int tile = s_tile;
    const int i0 = tile * kScanBlock * kScanItems + threadIdx.x * kScanItems;
    int v[kScanItems];
    int sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        v[j] = (i0 + j < n) ? in[i0 + j] : 0;
        sum += v[j];
    }
    // block exclusive scan of the per-thread sums
    int lane = __lane_id(), w = threadIdx.x / 64;
    int x = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_wave[w] = x;
    __syncthreads();
    int wave_off = 0, total = 0;
    for (int k = 0; k < kScanBlock / 64; k++) {
        if (k < w) wave_off += s_wave[k];
        total += s_wave[k];
    }
    int excl = wave_off + x - sum;
    if (threadIdx.x == 0) {
        int prefix = 0;
        if (tile == 0) {
            __hip_atomic_store(&status[0], kScanInc | (uint32_t)total, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&status[tile], kScanAgg | (uint32_t)total, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            int k = tile - 1, spins = 0;
            while (k >= 0) {
                uint64_t st = __hip_atomic_load(&status[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                uint64_t flag = st & (3ull << 62);
                if (flag == 0ull) {
                    if (++spins > (1 << 26)) {
                        atomicMin(err, err_key(0, -10));
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                prefix += (int)(uint32_t)st;
                if (flag == kScanInc) break;
                --k;
            }
            __hip_atomic_store(&status[tile], kScanInc | (uint32_t)(prefix + total), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        s_prefix = prefix;
    }
    __syncthreads();
    int run = s_prefix + excl;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        if (i0 + j < n) out[i0 + j] = run;
        run += v[j];
    }
    const int last_tile = (n + kScanBlock * kScanItems - 1) / (kScanBlock * kScanItems) - 1;
    if (tile == (last_tile < 0 ? 0 : last_tile) && threadIdx.x == kScanBlock - 1) out[n] = run;
}

// Slots within a vertex's bucket come in any order: the tile ranks its
// half-edges per vertex in LDS, reserves each vertex's run with one global
// atomic, and places them (the match does not depend on the order).
__global__ void __launch_bounds__(256) k_bucket(const int32_t *__restrict__ org, int nh,
                                                const int32_t *__restrict__ vstart, int32_t *fill, int2 *bucket) {
    __shared__ int s_hist[kHistBins];
    __shared__ int s_lohi[2];
    const int TB = 256 * kTileItems;
    for (int base = blockIdx.x * TB; base < nh; base += gridDim.x * TB) {   // block-uniform
        int v[kTileItems], w[kTileItems];
        int vlo = 0x7fffffff, vhi = -1;
#pragma unroll
        for (int j = 0; j < kTileItems; j++) {
            const int h = base + j * 256 + threadIdx.x;
            v[j] = -1;
            if (h < nh) {
                v[j] = org[h];
                w[j] = org[he_next_b(h)];
                vlo = min(vlo, v[j]);
                vhi = max(vhi, v[j]);
            }
        }
        int lo, hi;
        block_range(vlo, vhi, s_lohi, lo, hi);
        if (hi >= lo && hi - lo < kHistBins) {   // block-uniform
            const int range = hi - lo + 1;
            for (int k = threadIdx.x; k < range; k += 256) s_hist[k] = 0;
            __syncthreads();
            int rank[kTileItems];
#pragma unroll
            for (int j = 0; j < kTileItems; j++) rank[j] = v[j] >= 0 ? atomicAdd(&s_hist[v[j] - lo], 1) : 0;
            __syncthreads();
            for (int k = threadIdx.x; k < range; k += 256) {
                const int n = s_hist[k];
                if (n) s_hist[k] = atomicAdd(&fill[lo + k], n);   // the run's first slot in the bucket
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kTileItems; j++)
                if (v[j] >= 0)
                    bucket[vstart[v[j]] + s_hist[v[j] - lo] + rank[j]] = make_int2(base + j * 256 + threadIdx.x, w[j]);
        } else {
#pragma unroll
            for (int j = 0; j < kTileItems; j++)
                if (v[j] >= 0)
                    bucket[vstart[v[j]] + atomicAdd(&fill[v[j]], 1)] = make_int2(base + j * 256 + threadIdx.x, w[j]);
        }
        __syncthreads();   // the histogram and range are reused by the next tile
    }
}

__global__ void k_match(const int32_t *__restrict__ org, int nt, const int32_t *__restrict__ vstart,
                        const int2 *__restrict__ bucket, int32_t *__restrict__ twin,
                        unsigned long long *err) {
    const int nh = 3 * nt;
    for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < nh; h += gridDim.x * blockDim.x) {
        int u = org[h], v = org[he_next_b(h)];
        int found = -1, nrev = 0, ndup = 0;
        for (int k = vstart[v], e = vstart[v + 1]; k < e; k++) {
            const int2 g = bucket[k];   // (half-edge v->w, w)
            if (g.y == u) {
                found = g.x;
                ++nrev;
            }
        }
        // a second u->v: when some v->u exists, its own search finds both
        // u->v and reports them, so only a half-edge without a reverse looks
        if (nrev == 0) {
            for (int k = vstart[u], e = vstart[u + 1]; k < e; k++) {
                const int2 g = bucket[k];
                if (g.x != h && g.y == v) ++ndup;
            }
        }
        if (nrev > 1 || ndup > 0) atomicMin(err, err_key(1ull + nt + h, -4));
        twin[h] = nrev == 1 ? found : -1;
    }
}


// ---------------------------------------------------------------------------
// compact half-edge encoding
// ---------------------------------------------------------------------------

// 16-bit offset of v from base, or kEsc16 when it does not fit (or is 0 and
// zero is reserved: twins, where 0 means boundary).
__device__ __forceinline__ int off16(int v, int base, bool zero_reserved) {
    const int d = v - base;
    return (d > kEsc16 && d <= 32767 && !(zero_reserved && d == 0)) ? d : kEsc16;
}

// One thread per triangle: its record and its three twin offsets; the
// escapes are counted (one atomic per wave that has any).
__global__ void __launch_bounds__(256) k_compact_encode(const int32_t *__restrict__ org,
                                                        const int32_t *__restrict__ twin, int nt, int2 *org8,
                                                        int16_t *twin16, int32_t *nesc) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int n = 0;
    if (t < nt) {
        const int v0 = org[3 * t], v1 = org[3 * t + 1], v2 = org[3 * t + 2];
        const int d1 = off16(v1, v0, false), d2 = off16(v2, v0, false);
        n += (d1 == kEsc16) + (d2 == kEsc16);
        org8[t] = make_int2(v0, (d1 & 0xffff) | (d2 << 16));
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const int h = 3 * t + i, g = twin[h];
            const int d = g < 0 ? 0 : off16(g, h, true);
            n += d == kEsc16;
            twin16[h] = (int16_t)d;
        }
    }
    const unsigned long long any = __ballot(n != 0);
    if (any) {
        int w = n;
        for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o);
        if (__lane_id() == __ffsll((long long)any) - 1) atomicAdd(nesc, w);
    }
}

__device__ __forceinline__ void esc_insert(int32_t *esc, int32_t mask, int32_t key, int32_t val) {
    uint32_t slot = esc_hash(key) & (uint32_t)mask;
    for (int k = 0; k <= mask; k++) {
        const int32_t prev = atomicCAS(esc + 2 * slot, kEscEmpty, key);
        if (prev == kEscEmpty || prev == key) {
            esc[2 * slot + 1] = val;
            return;
        }
        slot = (slot + 1) & (uint32_t)mask;
    }
}

__global__ void k_esc_clear(int32_t *esc, int n) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
        esc[k] = (k & 1) ? 0 : kEscEmpty;
}

// Every value the encoder could not fit goes into the table.
__global__ void __launch_bounds__(256) k_compact_escapes(const int32_t *__restrict__ org,
                                                         const int32_t *__restrict__ twin, int nt, int32_t *esc,
                                                         int32_t mask) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const int v0 = org[3 * t];
#pragma unroll
    for (int i = 1; i < 3; i++) {
        const int v = org[3 * t + i];
        if (off16(v, v0, false) == kEsc16) esc_insert(esc, mask, ~(3 * t + i), v);
    }
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const int h = 3 * t + i, g = twin[h];
        if (g >= 0 && off16(g, h, true) == kEsc16) esc_insert(esc, mask, h, g);
    }
}

__device__ __forceinline__ int32_t esc_get(const int32_t *esc, int32_t mask, int32_t key) {
    uint32_t slot = esc_hash(key) & (uint32_t)mask;
    for (int k = 0; k <= mask; k++) {
        const int32_t kk = esc[2 * slot];
        if (kk == key) return esc[2 * slot + 1];
        if (kk == kEscEmpty) break;
        slot = (slot + 1) & (uint32_t)mask;
    }
    return -1;
}

__global__ void __launch_bounds__(256) k_compact_decode(const int2 *__restrict__ org8,
                                                        const int16_t *__restrict__ twin16,
                                                        const int32_t *__restrict__ esc, int32_t mask, int nt,
                                                        int32_t *org, int32_t *twin) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const int2 r = org8[t];
    const int d[3] = {0, (int)(int16_t)(r.y & 0xffff), r.y >> 16};
    org[3 * t] = r.x;
#pragma unroll
    for (int i = 1; i < 3; i++) org[3 * t + i] = d[i] == kEsc16 ? esc_get(esc, mask, ~(3 * t + i)) : r.x + d[i];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const int h = 3 * t + i, v = twin16[h];
        twin[h] = v == 0 ? -1 : (v == kEsc16 ? esc_get(esc, mask, h) : h + v);
    }
}

inline int grid_for(long long n, int block, int cap = 1 << 16) {
    long long g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (int)(g > cap ? cap : g);
}

}  // namespace

int32_t build_scan_tiles(int32_t n) {
    int per = kScanBlock * kScanItems;
    int k = (n + per - 1) / per;
    return k < 1 ? 1 : k;
}

hipError_t launch_build_orient(const BuildBuffers &b, hipStream_t s) {
    hipLaunchKernelGGL(k_check_xy, dim3(grid_for(b.nv, 256)), dim3(256), 0, s, b.xy, b.nv, b.err_key);
    if (b.nt > 0)
        hipLaunchKernelGGL(k_orient, dim3(grid_for(b.nt, 256 * kTileItems)), dim3(256), 0, s, b.xy, b.tri, b.nv, b.nt,
                           b.org, b.deg, b.err_key, b.nflipped);
    return hipGetLastError();
}

hipError_t launch_build_link(const BuildBuffers &b, hipStream_t s) {
    int tiles = build_scan_tiles(b.nv);
    hipLaunchKernelGGL(k_scan_excl, dim3(tiles), dim3(kScanBlock), 0, s, b.deg, b.vstart, b.nv,
                       b.scan_status, b.scan_ctr, b.err_key);
    long long nh = 3ll * b.nt;
    if (nh > 0) {
        hipLaunchKernelGGL(k_bucket, dim3(grid_for(nh, 256 * kTileItems)), dim3(256), 0, s, b.org, (int)nh, b.vstart,
                           b.fill, b.bucket);
        hipLaunchKernelGGL(k_match, dim3(grid_for(nh, 256)), dim3(256), 0, s, b.org, b.nt, b.vstart,
                           b.bucket, b.twin, b.err_key);
    }
    return hipGetLastError();
}

hipError_t launch_compact_encode(const CompactBuffers &c, hipStream_t s) {
    if (c.nt > 0)
        hipLaunchKernelGGL(k_compact_encode, dim3((c.nt + 255) / 256), dim3(256), 0, s, c.org, c.twin, c.nt, c.org8,
                           c.twin16, c.nesc);
    return hipGetLastError();
}

hipError_t launch_compact_escapes(const CompactBuffers &c, hipStream_t s) {
    const long long n = 2ll * ((long long)c.esc_mask + 1);
    hipLaunchKernelGGL(k_esc_clear, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, c.esc, (int)n);
    if (c.nt > 0)
        hipLaunchKernelGGL(k_compact_escapes, dim3((c.nt + 255) / 256), dim3(256), 0, s, c.org, c.twin, c.nt, c.esc,
                           c.esc_mask);
    return hipGetLastError();
}

hipError_t launch_compact_decode(const CompactBuffers &c, int32_t *org, int32_t *twin, hipStream_t s) {
    if (c.nt > 0)
        hipLaunchKernelGGL(k_compact_decode, dim3((c.nt + 255) / 256), dim3(256), 0, s, c.org8, c.twin16, c.esc,
                           c.esc_mask, c.nt, org, twin);
    return hipGetLastError();
}

}  // namespace gp
