// Reference light tree (section 3: one binary tree over all lights, lights
// stored in tree order; section 3.1: a simple LBVH over the light positions)
// and the breadth-first initial cut.
//
// Morton codes of the vertex sums (10 bits per axis, x most significant) are
// sorted with a stable LSD radix sort (ties keep input order), the binary
// radix tree over the sorted codes is built with one thread per internal
// node (Karras, "Maximizing parallelism in the construction of BVHs, octrees
// and k-d trees", HPG 2012), and the emitter records are gathered into tree
// order as 64-byte rows.
#include "rlc_internal.h"

namespace rlc {

namespace {

constexpr int kBlock = 256;
constexpr int kSortItems = 4;                       // keys per thread per tile
constexpr int kTile = kBlock * kSortItems;          // keys per tile
constexpr int kRadix = 256;

__global__ void __launch_bounds__(kBlock) k_tri_prep(const float* __restrict__ tri, uint32_t N,
                                                     float* __restrict__ sums, float* part_lo, float* part_hi,
                                                     uint32_t* err) {
    __shared__ float s_lo[3][kBlock];
    __shared__ float s_hi[3][kBlock];
    float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock) {
        const float* t = tri + 9 * i;
        bool finite = true;
        for (int k = 0; k < 9; ++k) finite &= fabsf(t[k]) <= 3.402823466e38f;
        if (!finite) atomicOr(err, RLC_DERR_INPUT);
        for (int a = 0; a < 3; ++a) {
            float v = (t[a] + t[3 + a]) + t[6 + a];
            sums[3 * i + a] = v;
            lo[a] = v < lo[a] ? v : lo[a];
            hi[a] = v > hi[a] ? v : hi[a];
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

// bbox[0..2] = lo, bbox[3..5] = hi, bbox[6..8] = 1024 / (hi - lo) (0 if flat)
__global__ void k_bbox_final(const float* part_lo, const float* part_hi, uint32_t nparts, float* bbox) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int a = 0; a < 3; ++a) {
        float lo = part_lo[a], hi = part_hi[a];
        for (uint32_t p = 1; p < nparts; ++p) {
            float l2 = part_lo[3 * p + a], h2 = part_hi[3 * p + a];
            lo = l2 < lo ? l2 : lo;
            hi = h2 > hi ? h2 : hi;
        }
        bbox[a] = lo;
        bbox[3 + a] = hi;
        bbox[6 + a] = (hi == lo) ? 0.0f : 1024.0f / (hi - lo);
    }
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void __launch_bounds__(kBlock) k_morton(const float* __restrict__ sums, const float* __restrict__ bbox,
                                                   uint32_t N, uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals) {
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        float v = floorf((sums[3 * i + a] - bbox[a]) * bbox[6 + a]);
        if (v > 1023.0f) v = 1023.0f;
        q[a] = (uint32_t)v;
    }
    keys[i] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    vals[i] = (uint32_t)i;
}

// ---- LSD radix sort: per pass a tile histogram, one exclusive scan over the
// digit-major histogram, and a stable scatter ranked inside each tile ----
__global__ void __launch_bounds__(kBlock) k_rs_hist(const uint32_t* __restrict__ keys, uint32_t N, int shift,
                                                    uint32_t ntiles, uint32_t* __restrict__ hist) {
    __shared__ uint32_t s_cnt[kRadix];
    s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    size_t base = (size_t)blockIdx.x * kTile;
    for (int r = 0; r < kSortItems; ++r) {
        size_t i = base + (size_t)r * kBlock + threadIdx.x;
        if (i < N) atomicAdd(&s_cnt[(keys[i] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * ntiles + blockIdx.x] = s_cnt[threadIdx.x];
}

__global__ void __launch_bounds__(kBlock) k_rs_scatter(const uint32_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ vals, uint32_t N, int shift,
                                                       uint32_t ntiles, const uint32_t* __restrict__ offs,
                                                       uint32_t* __restrict__ keys_out,
                                                       uint32_t* __restrict__ vals_out) {
    constexpr int kWaves = kBlock / 64;
    __shared__ uint32_t s_base[kRadix];            // running position per digit in this tile
    __shared__ uint32_t s_wcnt[kWaves][kRadix];    // per-wave digit counts of the current round
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    s_base[threadIdx.x] = offs[(size_t)threadIdx.x * ntiles + blockIdx.x];
    size_t base = (size_t)blockIdx.x * kTile;
    const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64u - lane));
    for (int r = 0; r < kSortItems; ++r) {
        for (int w = 0; w < kWaves; ++w) s_wcnt[w][threadIdx.x] = 0u;
        __syncthreads();
        size_t i = base + (size_t)r * kBlock + threadIdx.x;
        bool valid = i < N;
        uint32_t key = valid ? keys[i] : 0u;
        uint32_t digit = (key >> shift) & 0xFFu;
        // lanes of this wave holding the same digit
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            unsigned long long m = __ballot(((digit >> b) & 1u) != 0u);
            peers &= ((digit >> b) & 1u) ? m : ~m;
        }
        uint32_t rank_in_wave = (uint32_t)__popcll(peers & lt_mask);
        if (valid && rank_in_wave == 0u) s_wcnt[wave][digit] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = s_base[digit] + rank_in_wave;
            for (uint32_t w = 0; w < wave; ++w) pos += s_wcnt[w][digit];
            keys_out[pos] = key;
            vals_out[pos] = vals[i];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kWaves; ++w) add += s_wcnt[w][threadIdx.x];
        s_base[threadIdx.x] += add;
        __syncthreads();
    }
}

// Exclusive scan of n u32, in tiles of kScanTile = 1024 entries (256
// threads x 4, each thread's four loaded as one uint4 when aligned): the
// tiles' sums, their exclusive scan (the same three steps, recursively),
// then every tile's scan from its offset.  All loads are coalesced.
constexpr int kScanThreads = 256;
constexpr int kScanTile = 4 * kScanThreads;

// Inclusive scan of one value per thread over the block; returns the
// block's total in *total.
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t v, uint32_t* s_wave, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    if (lane == 63) s_wave[wave] = v;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        const uint32_t t = s_wave[w];
        before += w < wave ? t : 0u;
        all += t;
    }
    *total = all;
    return v + before;
}

// Four consecutive entries from i0 (a multiple of 4) as one uint4 when they
// are all in range and 16-byte aligned (a recursive level's scratch may not
// be), else one by one.
__device__ __forceinline__ bool vec4_ok(const uint32_t* data, size_t n, size_t i0) {
    return i0 + 3 < n && (reinterpret_cast<uintptr_t>(data + i0) & 15u) == 0;
}

__device__ __forceinline__ void load_tile(const uint32_t* data, size_t n, size_t i0, uint32_t x[4]) {
    if (vec4_ok(data, n, i0)) {
        const uint4 q = *reinterpret_cast<const uint4*>(data + i0);
        x[0] = q.x, x[1] = q.y, x[2] = q.z, x[3] = q.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = i0 + j < n ? data[i0 + j] : 0u;
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(const uint32_t* __restrict__ data, uint32_t n,
                                                            uint32_t* __restrict__ sums) {
    __shared__ uint32_t s_wave[kScanThreads / 64];
    const size_t i0 = (size_t)blockIdx.x * kScanTile + 4u * threadIdx.x;
    uint32_t x[4];
    load_tile(data, n, i0, x);
    uint32_t total;
    block_inclusive_scan((x[0] + x[1]) + (x[2] + x[3]), s_wave, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// offsets: exclusive scan of the tiles' sums, or null for a single tile.
__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(uint32_t* data, uint32_t n,
                                                             const uint32_t* __restrict__ offsets) {
    __shared__ uint32_t s_wave[kScanThreads / 64];
    const size_t i0 = (size_t)blockIdx.x * kScanTile + 4u * threadIdx.x;
    uint32_t x[4];
    load_tile(data, n, i0, x);
    const uint32_t mine = (x[0] + x[1]) + (x[2] + x[3]);
    uint32_t total;
    uint32_t run = block_inclusive_scan(mine, s_wave, &total) - mine;
    if (offsets) run += offsets[blockIdx.x];
    uint32_t y[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        y[j] = run;
        run += x[j];
    }
    if (vec4_ok(data, n, i0)) {
        *reinterpret_cast<uint4*>(data + i0) = make_uint4(y[0], y[1], y[2], y[3]);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (i0 + j < n) data[i0 + j] = y[j];
    }
}

__global__ void __launch_bounds__(kBlock) k_gather_records(const float* __restrict__ tri,
                                                           const float* __restrict__ emit,
                                                           const uint32_t* __restrict__ perm, uint32_t N,
                                                           float4* __restrict__ rec) {
    size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= N) return;
    size_t i = perm[j];
    const float* t = tri + 9 * i;
    float e1x = t[3] - t[0], e1y = t[4] - t[1], e1z = t[5] - t[2];
    float e2x = t[6] - t[0], e2y = t[7] - t[1], e2z = t[8] - t[2];
    float cx = e1y * e2z - e1z * e2y;
    float cy = e1z * e2x - e1x * e2z;
    float cz = e1x * e2y - e1y * e2x;
    float len = sqrtf((cx * cx + cy * cy) + cz * cz);
    float area = 0.0f, nx = 0.0f, ny = 0.0f, nz = 0.0f;
    if (len != 0.0f) {
        float inv = 1.0f / len;
        area = 0.5f * len;
        nx = cx * inv;
        ny = cy * inv;
        nz = cz * inv;
    }
    rec[4 * j + 0] = make_float4(t[0], t[1], t[2], t[3]);
    rec[4 * j + 1] = make_float4(t[4], t[5], t[6], t[7]);
    rec[4 * j + 2] = make_float4(t[8], emit[3 * i], emit[3 * i + 1], emit[3 * i + 2]);
    rec[4 * j + 3] = make_float4(area, nx, ny, nz);
}

// rank[perm[j]] = j: the sorted position of each input light.
__global__ void __launch_bounds__(kBlock) k_invert_perm(const uint32_t* __restrict__ perm, uint32_t N,
                                                        uint32_t* __restrict__ rank) {
    const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (j < N) rank[perm[j]] = (uint32_t)j;
}

// New emission of every light: input light i (read in input order, so the
// loads are coalesced and independent) into its record at sorted position
// rank[i] (one 12-byte store per light).
__global__ void __launch_bounds__(kBlock) k_scatter_emission(const float* __restrict__ emit,
                                                             const uint32_t* __restrict__ rank, uint32_t N,
                                                             float4* __restrict__ rec) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    const size_t j = rank[i];
    float* r = reinterpret_cast<float*>(rec + 4 * j + 2);
    r[1] = emit[3 * i];
    r[2] = emit[3 * i + 1];
    r[3] = emit[3 * i + 2];
}

// 64-bit key of sorted position j: (Morton << 32) | input index, all distinct
__device__ __forceinline__ int delta(const uint32_t* morton, const uint32_t* perm, int N, int i, int j) {
    if (j < 0 || j >= N) return -1;
    unsigned long long a = ((unsigned long long)morton[i] << 32) | perm[i];
    unsigned long long b = ((unsigned long long)morton[j] << 32) | perm[j];
    return __clzll((long long)(a ^ b));
}

__global__ void __launch_bounds__(kBlock) k_radix_tree(const uint32_t* __restrict__ morton,
                                                       const uint32_t* __restrict__ perm, uint32_t N,
                                                       uint32_t* __restrict__ left, uint32_t* __restrict__ right,
                                                       uint32_t* __restrict__ parent, uint32_t* __restrict__ first,
                                                       uint32_t* __restrict__ last, uint32_t* __restrict__ inode) {
    size_t gi = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int n = (int)N;
    if (gi < N) {  // leaves
        first[N - 1 + gi] = (uint32_t)gi;
        last[N - 1 + gi] = (uint32_t)gi;
    }
    if (gi == 0) {
        parent[0] = RLC_NONE;
        if (N > 1) inode[3] = RLC_NONE;
    }
    if (gi + 1 >= N) return;
    const int i = (int)gi;
    // direction of the range from the larger common prefix
    const int d = (delta(morton, perm, n, i, i + 1) - delta(morton, perm, n, i, i - 1)) > 0 ? 1 : -1;
    const int dmin = delta(morton, perm, n, i, i - d);
    int lmax = 2;
    while (delta(morton, perm, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(morton, perm, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = delta(morton, perm, n, i, j);
    // split: last position that still shares more than dnode bits with i
    int s = 0;
    for (int t = (l + 1) >> 1;; t = (t + 1) >> 1) {
        if (s + t <= l && delta(morton, perm, n, i, i + (s + t) * d) > dnode) s += t;
        if (t == 1) break;
    }
    const int gamma = i + s * d + (d < 0 ? -1 : 0);
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    const uint32_t lc = (lo == gamma) ? (N - 1u + (uint32_t)gamma) : (uint32_t)gamma;
    const uint32_t rc = (hi == gamma + 1) ? (N - 1u + (uint32_t)(gamma + 1)) : (uint32_t)(gamma + 1);
    left[i] = lc;
    right[i] = rc;
    parent[lc] = (uint32_t)i;
    parent[rc] = (uint32_t)i;
    first[i] = (uint32_t)lo;
    last[i] = (uint32_t)hi;
    inode[4 * i] = lc;
    inode[4 * i + 1] = rc;
    inode[4 * i + 2] = (uint32_t)(gamma + 1);
    if (lc + 1u < N) inode[4 * lc + 3] = (uint32_t)i;
    if (rc + 1u < N) inode[4 * rc + 3] = (uint32_t)i;
}

// Breadth-first initial cut, built once by one thread (setup).
__global__ void k_initial_cut(DevTree tree, uint32_t M, uint32_t* node, uint32_t* end, float* Qt, float* C) {
    __shared__ uint32_t list[2 * RLC_MMAX];
    __shared__ uint8_t gone[2 * RLC_MMAX];
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t N = tree.N;
    const uint32_t target = M < N ? M : N;
    uint32_t len = 1, live = 1, cursor = 0;
    list[0] = 0u;  // root (with one light, node 0 is that light's leaf)
    gone[0] = 0;
    while (live < target) {
        // earliest-enqueued node still in the list that has children
        while (cursor < len && (gone[cursor] || list[cursor] >= N - 1u)) ++cursor;
        if (cursor == len) break;
        uint32_t nd = list[cursor];
        gone[cursor] = 1;
        list[len] = tree.left[nd];
        gone[len++] = 0;
        list[len] = tree.right[nd];
        gone[len++] = 0;
        ++live;
    }
    uint32_t m = 0;
    for (uint32_t i = 0; i < len; ++i)
        if (!gone[i]) list[m++] = list[i];  // m <= i, safe in place
    for (uint32_t i = 1; i < m; ++i) {     // order by first light
        uint32_t v = list[i], j = i;
        while (j > 0 && tree.first[list[j - 1]] > tree.first[v]) {
            list[j] = list[j - 1];
            --j;
        }
        list[j] = v;
    }
    float acc = 0.0f;
    for (uint32_t s = 0; s < m; ++s) {
        node[s] = list[s];
        end[s] = tree.last[list[s]] + 1u;
        Qt[s] = 1.0f;
        acc = s ? acc + 1.0f : 1.0f;
        C[s] = acc;
    }
}

__global__ void k_check_finite(const float* __restrict__ a, uint32_t n, uint32_t* err) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(fabsf(a[i]) <= 3.402823466e38f)) atomicOr(err, RLC_DERR_INPUT);
}

__global__ void k_check_nonneg(const float* __restrict__ a, uint32_t n, uint32_t* err) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(a[i] >= 0.0f && a[i] <= 3.402823466e38f)) atomicOr(err, RLC_DERR_INPUT);
}

__global__ void k_fill_u32(uint32_t* a, uint32_t v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        a[i] = v;
}

__global__ void k_fill_u64(unsigned long long* a, unsigned long long v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        a[i] = v;
}

inline uint32_t blocks_for(size_t n, int b = kBlock) { return (uint32_t)((n + b - 1) / b); }

}  // namespace

hipError_t launch_tri_prep(const float* tri, uint32_t N, float* sums, float* part_lo, float* part_hi,
                           uint32_t nblocks, uint32_t* err, hipStream_t s) {
    hipLaunchKernelGGL(k_tri_prep, dim3(nblocks), dim3(kBlock), 0, s, tri, N, sums, part_lo, part_hi, err);
    return hipGetLastError();
}

hipError_t launch_bbox_final(const float* part_lo, const float* part_hi, uint32_t nparts, float* bbox,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, s, part_lo, part_hi, nparts, bbox);
    return hipGetLastError();
}

hipError_t launch_morton(const float* sums, const float* bbox, uint32_t N, uint32_t* keys, uint32_t* vals,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_morton, dim3(blocks_for(N)), dim3(kBlock), 0, s, sums, bbox, N, keys, vals);
    return hipGetLastError();
}

size_t scan_scratch_entries(size_t n) {
    size_t total = 0;
    while (n > (size_t)kScanTile) {
        n = (n + kScanTile - 1) / kScanTile;
        total += n;
    }
    return total;
}

// The histogram, then the scratch of its scan.
size_t radix_sort_hist_entries(uint32_t N) {
    const size_t h = (size_t)kRadix * blocks_for(N, kTile);
    return h + scan_scratch_entries(h);
}

hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp,
                            uint32_t* hist, uint32_t N, int bits, hipStream_t s) {
    uint32_t ntiles = blocks_for(N, kTile);
    uint32_t* kin = keys;
    uint32_t* vin = vals;
    uint32_t* kout = keys_tmp;
    uint32_t* vout = vals_tmp;
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist, dim3(ntiles), dim3(kBlock), 0, s, kin, N, shift, ntiles, hist);
        (void)launch_exclusive_scan(hist, (uint32_t)(ntiles * kRadix), hist + (size_t)ntiles * kRadix, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(kBlock), 0, s, kin, vin, N, shift, ntiles, hist, kout,
                           vout);
        uint32_t* t = kin;
        kin = kout;
        kout = t;
        t = vin;
        vin = vout;
        vout = t;
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && kin != keys) {
        e = hipMemcpyAsync(keys, kin, sizeof(uint32_t) * N, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(vals, vin, sizeof(uint32_t) * N, hipMemcpyDeviceToDevice, s);
    }
    return e;
}

hipError_t launch_exclusive_scan(uint32_t* data, uint32_t n, uint32_t* scratch, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t tiles = (uint32_t)((n + kScanTile - 1) / kScanTile);
    if (tiles == 1) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, data, n, (const uint32_t*)nullptr);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_sums, dim3(tiles), dim3(kScanThreads), 0, s, data, n, scratch);
    hipError_t e = launch_exclusive_scan(scratch, tiles, scratch + tiles, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kScanThreads), 0, s, data, n, scratch);
    return hipGetLastError();
}

hipError_t launch_gather_records(const float* tri, const float* emit, const uint32_t* perm, uint32_t N,
                                 float4* rec, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_records, dim3(blocks_for(N)), dim3(kBlock), 0, s, tri, emit, perm, N, rec);
    return hipGetLastError();
}

hipError_t launch_invert_perm(const uint32_t* perm, uint32_t N, uint32_t* rank, hipStream_t s) {
    hipLaunchKernelGGL(k_invert_perm, dim3(blocks_for(N)), dim3(kBlock), 0, s, perm, N, rank);
    return hipGetLastError();
}

hipError_t launch_scatter_emission(const float* emit, const uint32_t* rank, uint32_t N, float4* rec,
                                   hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_emission, dim3(blocks_for(N)), dim3(kBlock), 0, s, emit, rank, N, rec);
    return hipGetLastError();
}

hipError_t launch_radix_tree(const uint32_t* morton, const uint32_t* perm, uint32_t N, uint32_t* left,
                             uint32_t* right, uint32_t* parent, uint32_t* first, uint32_t* last, uint32_t* inode,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_radix_tree, dim3(blocks_for(N)), dim3(kBlock), 0, s, morton, perm, N, left, right, parent,
                       first, last, inode);
    return hipGetLastError();
}

hipError_t launch_initial_cut(DevTree tree, uint32_t M, uint32_t* node, uint32_t* end, float* Qt, float* C,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_initial_cut, dim3(1), dim3(64), 0, s, tree, M, node, end, Qt, C);
    return hipGetLastError();
}

hipError_t launch_check_finite(const float* a, uint32_t n, uint32_t* err, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_finite, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, n, err);
    return hipGetLastError();
}

hipError_t launch_check_nonneg(const float* a, uint32_t n, uint32_t* err, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_nonneg, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, n, err);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* a, uint32_t v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint32_t nb = blocks_for(n);
    if (nb > 16384u) nb = 16384u;
    hipLaunchKernelGGL(k_fill_u32, dim3(nb), dim3(kBlock), 0, s, a, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* a, unsigned long long v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint32_t nb = blocks_for(n);
    if (nb > 16384u) nb = 16384u;
    hipLaunchKernelGGL(k_fill_u64, dim3(nb), dim3(kBlock), 0, s, a, v, n);
    return hipGetLastError();
}

}  // namespace rlc
