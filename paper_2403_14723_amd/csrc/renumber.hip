// Optional renumbering of a triangulation along a Z-order (Morton) curve, run
// on the device before the half-edge build (GP_RENUMBER).
//
// The meshing kernels read neighbours' labels, twins and next' by index, so
// they run fastest when neighbouring triangles have nearby indices.  Meshes
// numbered without locality (a Delaunay triangulator's output order, a
// shuffled file) are renumbered here: vertices in the Morton order of their
// coordinates, triangles in the Morton order of their centroids (corner order
// within a triangle kept).  The new-to-old maps are kept with the mesh.
#include <hipcub/hipcub.hpp>

#include "gp_internal.h"

namespace gp {

namespace {

// The 31 low bits of v spread to the even bits of a 64-bit word.
__device__ __forceinline__ uint64_t spread31(uint32_t v) {
    uint64_t x = v & 0x7fffffffu;
    x = (x | (x << 16)) & 0x0000ffff0000ffffull;
    x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
    x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

// Morton code of (x, y), coordinates clamped to [0, 2^31) (valid inputs are
// in [0, 2^30]; others are reported by the build later).
__device__ __forceinline__ uint64_t morton(long long x, long long y) {
    const uint32_t cx = (uint32_t)(x < 0 ? 0 : (x > 0x7fffffff ? 0x7fffffff : x));
    const uint32_t cy = (uint32_t)(y < 0 ? 0 : (y > 0x7fffffff ? 0x7fffffff : y));
    return spread31(cx) | (spread31(cy) << 1);
}

__global__ void k_vertex_keys(const int2 *__restrict__ xy, int nv, uint64_t *keys, int32_t *vals) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int2 p = xy[v];
    keys[v] = morton(p.x, p.y);
    vals[v] = v;
}

// vinv: old -> new vertex index; xy_out in the new order.
__global__ void k_vertex_gather(const int2 *__restrict__ xy, const int32_t *__restrict__ vperm, int nv,
                                int32_t *vinv, int2 *xy_out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nv) return;
    const int v = vperm[k];
    vinv[v] = k;
    xy_out[k] = xy[v];
}

// A triangle with an index outside [0, nv) gets the largest key (the build
// reports it later, wherever it lands).
__global__ void k_triangle_keys(const int2 *__restrict__ xy, const int32_t *__restrict__ tri, int nv, int nt,
                                uint64_t *keys, int32_t *vals) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    long long sx = 0, sy = 0;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const int v = tri[3 * t + i];
        if (v >= 0 && v < nv) {
            const int2 p = xy[v];
            sx += p.x;
            sy += p.y;
        } else {
            ok = false;
        }
    }
    keys[t] = ok ? morton(sx / 3, sy / 3) : ~0ull;
    vals[t] = t;
}

// Triangles in the new order with new vertex indices (invalid ones kept).
__global__ void k_triangle_gather(const int32_t *__restrict__ tri, const int32_t *__restrict__ tperm,
                                  const int32_t *__restrict__ vinv, int nv, int nt, int32_t *tri_out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    const int t = tperm[k];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const int v = tri[3 * t + i];
        tri_out[3 * k + i] = (v >= 0 && v < nv) ? vinv[v] : v;
    }
}

inline int blocks_for(int n) { return n > 0 ? (n + 255) / 256 : 1; }

}  // namespace

size_t renumber_sort_bytes(int32_t n) {
    size_t b = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                           (const int32_t *)nullptr, (int32_t *)nullptr, n < 1 ? 1 : n, 0, 64,
                                           (hipStream_t)0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return b;
}

hipError_t launch_renumber(const RenumberBuffers &b, hipStream_t s) {
    hipError_t e = hipSuccess;
    size_t tb = b.sort_bytes;
    if (b.nv > 0) {
        hipLaunchKernelGGL(k_vertex_keys, dim3(blocks_for(b.nv)), dim3(256), 0, s, b.xy_in, b.nv, b.keys, b.vals);
        e = hipcub::DeviceRadixSort::SortPairs(b.sort_tmp, tb, b.keys, b.keys_alt, b.vals, b.vperm, b.nv, 0, 62, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_vertex_gather, dim3(blocks_for(b.nv)), dim3(256), 0, s, b.xy_in, b.vperm, b.nv, b.vinv,
                           b.xy_out);
    }
    if (b.nt > 0) {
        hipLaunchKernelGGL(k_triangle_keys, dim3(blocks_for(b.nt)), dim3(256), 0, s, b.xy_in, b.tri_in, b.nv, b.nt,
                           b.keys, b.vals);
        tb = b.sort_bytes;
        e = hipcub::DeviceRadixSort::SortPairs(b.sort_tmp, tb, b.keys, b.keys_alt, b.vals, b.tperm, b.nt, 0, 64, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_triangle_gather, dim3(blocks_for(b.nt)), dim3(256), 0, s, b.tri_in, b.tperm, b.vinv,
                           b.nv, b.nt, b.tri_out);
    }
    return hipGetLastError();
}

}  // namespace gp
