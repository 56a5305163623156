// Occluders for the shadow rays: box packing, a uniform grid over the boxes
// (counts, exclusive scan, fill), and a visibility-only kernel.
#include "rlc_internal.h"

namespace rlc {

namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_pack_boxes(const float* __restrict__ aabb, uint32_t K,
                                                       float4* __restrict__ box, float* part_lo, float* part_hi,
                                                       uint32_t* err) {
    __shared__ float s_lo[3][kBlock];
    __shared__ float s_hi[3][kBlock];
    float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < K; i += (size_t)gridDim.x * kBlock) {
        const float* a = aabb + 6 * i;
        bool ok = true;
        for (int k = 0; k < 6; ++k) ok &= fabsf(a[k]) <= 3.402823466e38f;
        for (int k = 0; k < 3; ++k) ok &= a[k] <= a[3 + k];
        if (!ok) atomicOr(err, RLC_DERR_INPUT);
        box[2 * i] = make_float4(a[0], a[1], a[2], a[3]);
        box[2 * i + 1] = make_float4(a[4], a[5], 0.0f, 0.0f);
        for (int k = 0; k < 3; ++k) {
            lo[k] = a[k] < lo[k] ? a[k] : lo[k];
            hi[k] = a[3 + k] > hi[k] ? a[3 + k] : hi[k];
        }
    }
    for (int a = 0; a < 3; ++a) {
        s_lo[a][threadIdx.x] = lo[a];
        s_hi[a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int a = 0; a < 3; ++a) {
                float l2 = s_lo[a][threadIdx.x + off], h2 = s_hi[a][threadIdx.x + off];
                if (l2 < s_lo[a][threadIdx.x]) s_lo[a][threadIdx.x] = l2;
                if (h2 > s_hi[a][threadIdx.x]) s_hi[a][threadIdx.x] = h2;
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) {
            part_lo[3 * blockIdx.x + a] = s_lo[a][0];
            part_hi[3 * blockIdx.x + a] = s_hi[a][0];
        }
}

__global__ void __launch_bounds__(kBlock) k_occ_count(const float4* __restrict__ box, uint32_t K, DevOcc occ,
                                                      uint32_t* __restrict__ counts) {
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= K) return;
    int lo[3], hi[3];
    box_cells(occ, box[2 * i], box[2 * i + 1], lo, hi);
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x)
                atomicAdd(&counts[(uint32_t)x + occ.res * ((uint32_t)y + occ.res * (uint32_t)z)], 1u);
}

// Space of cell c's list in ref: none for 0 or 1 box, count + indices otherwise.
__global__ void __launch_bounds__(kBlock) k_occ_sizes(const uint32_t* __restrict__ counts, uint32_t ncell,
                                                      uint32_t* __restrict__ sizes) {
    size_t c = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (c > ncell) return;
    uint32_t n = c < ncell ? counts[c] : 0u;
    sizes[c] = n >= 2u ? n + 1u : 0u;
}

__global__ void __launch_bounds__(kBlock) k_occ_heads(const uint32_t* __restrict__ counts,
                                                      const uint32_t* __restrict__ start, uint32_t ncell,
                                                      uint32_t* __restrict__ head, uint32_t* __restrict__ ref) {
    size_t c = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncell) return;
    uint32_t n = counts[c];
    if (n >= 2u) {
        head[c] = RLC_OCC_LIST | start[c];
        ref[start[c]] = n;
    } else {
        head[c] = 0u;  // a single box writes its own header in k_occ_fill
    }
}

__global__ void __launch_bounds__(kBlock) k_occ_fill(const float4* __restrict__ box, uint32_t K, DevOcc occ,
                                                     const uint32_t* __restrict__ counts,
                                                     const uint32_t* __restrict__ start,
                                                     uint32_t* __restrict__ cursor, uint32_t* __restrict__ head,
                                                     uint32_t* __restrict__ ref) {
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= K) return;
    int lo[3], hi[3];
    box_cells(occ, box[2 * i], box[2 * i + 1], lo, hi);
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
                uint32_t c = (uint32_t)x + occ.res * ((uint32_t)y + occ.res * (uint32_t)z);
                if (counts[c] == 1u)
                    head[c] = RLC_OCC_ONE | (uint32_t)i;
                else
                    ref[start[c] + 1u + atomicAdd(&cursor[c], 1u)] = (uint32_t)i;
            }
}

// Octant radii of the cells no box overlaps (the skip headers; see
// occ_trace.h).  For the octant with signs s, the distance from cell c to the
// nearest cell a box overlaps within that octant, D_s(c) = min over such
// cells c + (i s_x, j s_y, k s_z), i, j, k >= 0, of max(i, j, k), is
// separable: pass x takes, along the grid line through c, the nearest
// occupied cell at or ahead of c in direction s_x; pass y the minimum over
// j >= 0 of max(j, pass x at c + j s_y); pass z the same over k with pass y.
// Distances are capped at kFar = RLC_OCC_SKIP_MAX + 1, so each pass looks
// that far ahead.  Pass x keeps its two directions in 4-bit fields, pass y
// its four (x, y) sign pairs; pass z writes, into the header of each empty
// cell, the eight radii D_s(c) - 1 (3 bits each, octant o at bits 3o).
constexpr int kFar = (int)RLC_OCC_SKIP_MAX + 1;

__global__ void __launch_bounds__(kBlock) k_occ_skip(const uint32_t* __restrict__ src, uint32_t* dst, uint32_t res,
                                                     uint32_t axis) {
    const size_t c = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const size_t ncell = (size_t)res * res * res;
    if (c >= ncell) return;
    const size_t stride = axis == 0 ? 1 : (axis == 1 ? (size_t)res : (size_t)res * res);
    const int ca = (int)((c / stride) % res);
    const int nin = axis == 0 ? 1 : (axis == 1 ? 2 : 4);  // sign combinations of the earlier axes
    int best[8];
    for (int q = 0; q < 8; ++q) best[q] = kFar;
    for (int dir = 0; dir < 2; ++dir) {  // dir 1: this axis's sign is negative
        const int reach = dir ? ca : (int)res - 1 - ca;
        const int kmax = reach < kFar ? reach : kFar;
        for (int k = 0; k <= kmax; ++k) {
            const ptrdiff_t off = (ptrdiff_t)k * (ptrdiff_t)stride;
            const uint32_t v = src[(size_t)(dir ? (ptrdiff_t)c - off : (ptrdiff_t)c + off)];
            for (int q = 0; q < nin; ++q) {
                int e;
                if (axis == 0)
                    e = (v & (RLC_OCC_ONE | RLC_OCC_LIST)) ? k : kFar;
                else {
                    const int prev = (int)((v >> (4 * q)) & 15u);
                    e = k > prev ? k : prev;
                }
                const int slot = q + nin * dir;
                best[slot] = e < best[slot] ? e : best[slot];
            }
        }
    }
    if (axis < 2) {
        uint32_t w = 0;
        for (int q = 0; q < 2 * nin; ++q) w |= (uint32_t)best[q] << (4 * q);
        dst[c] = w;
    } else if (!(dst[c] & (RLC_OCC_ONE | RLC_OCC_LIST))) {
        uint32_t w = 0;
        for (int q = 0; q < 8; ++q) w |= (uint32_t)(best[q] - 1) << (3 * q);
        dst[c] = w;
    }
}

__global__ void __launch_bounds__(kBlock) k_visible(DevOcc occ, float t_lo, const float* __restrict__ x,
                                                    const float* __restrict__ y, uint32_t n,
                                                    uint8_t* __restrict__ vis) {
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    float o[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
    float d[3] = {y[3 * i] - o[0], y[3 * i + 1] - o[1], y[3 * i + 2] - o[2]};
    vis[i] = segment_blocked(occ, o, d, t_lo) ? 0 : 1;
}

inline uint32_t blocks_for(size_t n) { return (uint32_t)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_pack_boxes(const float* aabb, uint32_t K, float4* box, float* part_lo, float* part_hi,
                             uint32_t nblocks, uint32_t* err, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_boxes, dim3(nblocks), dim3(kBlock), 0, s, aabb, K, box, part_lo, part_hi, err);
    return hipGetLastError();
}

hipError_t launch_occ_count(const float4* box, uint32_t K, DevOcc occ, uint32_t* counts, hipStream_t s) {
    if (K == 0) return hipSuccess;
    hipLaunchKernelGGL(k_occ_count, dim3(blocks_for(K)), dim3(kBlock), 0, s, box, K, occ, counts);
    return hipGetLastError();
}

hipError_t launch_occ_lists(const float4* box, uint32_t K, DevOcc occ, const uint32_t* counts, uint32_t* start,
                            uint32_t* cursor, uint32_t* head, uint32_t* ref, hipStream_t s) {
    if (K == 0) return hipSuccess;
    const uint32_t ncell = occ.res * occ.res * occ.res;
    hipLaunchKernelGGL(k_occ_heads, dim3(blocks_for(ncell)), dim3(kBlock), 0, s, counts, start, ncell, head, ref);
    hipLaunchKernelGGL(k_occ_fill, dim3(blocks_for(K)), dim3(kBlock), 0, s, box, K, occ, counts, start, cursor, head,
                       ref);
    return hipGetLastError();
}

hipError_t launch_occ_skip(uint32_t* head, uint32_t* tmp0, uint32_t* tmp1, uint32_t res, hipStream_t s) {
    const size_t ncell = (size_t)res * res * res;
    if (ncell == 0) return hipSuccess;
    const dim3 grid(blocks_for(ncell));
    hipLaunchKernelGGL(k_occ_skip, grid, dim3(kBlock), 0, s, head, tmp0, res, 0u);
    hipLaunchKernelGGL(k_occ_skip, grid, dim3(kBlock), 0, s, tmp0, tmp1, res, 1u);
    hipLaunchKernelGGL(k_occ_skip, grid, dim3(kBlock), 0, s, tmp1, head, res, 2u);
    return hipGetLastError();
}

hipError_t launch_occ_sizes(const uint32_t* counts, uint32_t ncell, uint32_t* sizes, hipStream_t s) {
    hipLaunchKernelGGL(k_occ_sizes, dim3(blocks_for((size_t)ncell + 1)), dim3(kBlock), 0, s, counts, ncell, sizes);
    return hipGetLastError();
}

hipError_t launch_visible(DevOcc occ, float t_lo, const float* x, const float* y, uint32_t n, uint8_t* vis,
                          hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_visible, dim3(blocks_for(n)), dim3(kBlock), 0, s, occ, t_lo, x, y, n, vis);
    return hipGetLastError();
}

}  // namespace rlc
