// Per-frame kernels of the hot path: sample (section 3: cluster from the
// cell's cdf, light inside the cluster), shade (shadow ray, contribution,
// estimate), learn (fixed-point statistics for Eq. 1), and the fused kernel
// that runs all three for one sample per lane.
#include "rlc_internal.h"

namespace rlc {

namespace {

constexpr int kBlock = 256;
static_assert(kBlock == (int)RLC_FRAME_BLOCK, "fused kernel block size");

__device__ __forceinline__ bool pow2_le64(uint32_t spp) { return spp <= 64u && (spp & (spp - 1u)) == 0u; }

// Per-block merge of the (cell, cluster) statistics before the global
// atomics: the block's samples add their fixed-point reward and count into a
// small LDS hash table keyed by bin = cell * M + cluster (integer sums, so
// order-free), then each distinct bin is added to the cell table once.  A
// sample whose bin finds no slot within kAggProbes probes goes straight to
// the cell table.
constexpr uint32_t kNoBin = 0xFFFFFFFFu;
constexpr int kAggProbes = 32;

template <int SLOTS>
struct AggTableT {
    static_assert((SLOTS & (SLOTS - 1)) == 0, "power of two");
    uint32_t bin[SLOTS];
    unsigned long long sum[SLOTS];
    uint32_t cnt[SLOTS];
};
using AggTable = AggTableT<2 * kBlock>;

template <int SLOTS>
__device__ __forceinline__ void agg_clear(AggTableT<SLOTS>& t) {
    for (int j = threadIdx.x; j < SLOTS; j += kBlock) {
        t.bin[j] = kNoBin;
        t.sum[j] = 0ull;
        t.cnt[j] = 0u;
    }
}

template <int SLOTS>
__device__ __forceinline__ void agg_add(AggTableT<SLOTS>& t, const FrameParams& fp, uint32_t cell, uint32_t s,
                                        unsigned long long q) {
    if (cell == RLC_NONE) return;
    const uint32_t bin = cell * fp.cells.M + s;
    constexpr int kBits = __builtin_ctz(SLOTS);
    uint32_t h = (bin * 2654435761u) >> (32 - kBits);  // Fibonacci hash
    // kept as a loop: unrolled, its 32 exits nest 32 exec masks, which spill
    // to VGPR lanes and are read back on every pass through the exits
#pragma unroll 1
    for (int probe = 0; probe < kAggProbes; ++probe) {
        const uint32_t old = atomicCAS(&t.bin[h], kNoBin, bin);
        if (old == kNoBin || old == bin) {
            add_fixed(&t.sum[h], q, fp.err);
            atomicAdd(&t.cnt[h], 1u);
            return;
        }
        h = (h + 1u) & (SLOTS - 1);
    }
    add_fixed(&fp.cells.sum[bin], q, fp.err);
    atomicAdd(&fp.cells.cnt[bin], 1u);
}

// Each thread flushes and clears its own slots, so no barrier is needed
// between the two; the caller syncs before the table is used again.
template <int SLOTS>
__device__ __forceinline__ void agg_flush(AggTableT<SLOTS>& t, const FrameParams& fp) {
    for (int j = threadIdx.x; j < SLOTS; j += kBlock) {
        const uint32_t n = t.cnt[j];
        if (n) {
            const size_t idx = t.bin[j];
            add_fixed(&fp.cells.sum[idx], t.sum[j], fp.err);
            atomicAdd(&fp.cells.cnt[idx], n);
            t.bin[j] = kNoBin;
            t.sum[j] = 0ull;
            t.cnt[j] = 0u;
        }
    }
}

// A point's spp estimates summed one after another in sample order (the
// order of the definition), through LDS: the block's 256 samples hold whole
// points when spp is a power of two up to 64.
__device__ __forceinline__ void point_sums(float (*s_e)[3], const float e[3], uint32_t spp, bool valid, uint32_t k,
                                           uint32_t p, float* __restrict__ radiance) {
    const float inv_spp = 1.0f / (float)spp;
    s_e[threadIdx.x][0] = e[0];
    s_e[threadIdx.x][1] = e[1];
    s_e[threadIdx.x][2] = e[2];
    __syncthreads();
    if (valid && k == 0) {
        float acc[3] = {e[0], e[1], e[2]};
        for (uint32_t j = 1; j < spp; ++j) {
            acc[0] = acc[0] + s_e[threadIdx.x + j][0];
            acc[1] = acc[1] + s_e[threadIdx.x + j][1];
            acc[2] = acc[2] + s_e[threadIdx.x + j][2];
        }
        radiance[3 * (size_t)p] = acc[0] * inv_spp;
        radiance[3 * (size_t)p + 1] = acc[1] * inv_spp;
        radiance[3 * (size_t)p + 2] = acc[2] * inv_spp;
    }
}

__global__ void __launch_bounds__(kBlock) k_sample(FrameParams fp, const float* __restrict__ pos,
                                                   const float* __restrict__ nrm, uint32_t P, uint32_t spp,
                                                   uint32_t frame, rlc_samples out) {
    uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    size_t i = (size_t)b * kBlock + threadIdx.x;
    size_t n = (size_t)P * spp;
    if (i >= n) return;
    uint32_t p = (uint32_t)(i / spp), k = (uint32_t)(i % spp);
    Sample sm;
    const float x[3] = {pos[3 * (size_t)p], pos[3 * (size_t)p + 1], pos[3 * (size_t)p + 2]};
    float nn[3] = {0.0f, 0.0f, 0.0f};
    if (nrm) {
        nn[0] = nrm[3 * (size_t)p];
        nn[1] = nrm[3 * (size_t)p + 1];
        nn[2] = nrm[3 * (size_t)p + 2];
    }
    draw_sample(fp, x, nn, p, k, frame, sm);
    if (out.d_key) out.d_key[i] = sm.key;
    if (out.d_cell) out.d_cell[i] = sm.cell;
    if (out.d_ready) out.d_ready[i] = sm.ready;
    if (out.d_slot) out.d_slot[i] = sm.s;
    if (out.d_light) out.d_light[i] = sm.light;
    if (out.d_inv_pdf) out.d_inv_pdf[i] = sm.inv_pdf;
    if (out.d_comp) out.d_comp[i] = sm.comp;
    if (out.d_y) {
        out.d_y[3 * i] = sm.y[0];
        out.d_y[3 * i + 1] = sm.y[1];
        out.d_y[3 * i + 2] = sm.y[2];
    }
}

// One lane per sample; the spp samples of a point share aligned lanes.
__global__ void __launch_bounds__(kBlock) k_shade(FrameParams fp, const float* __restrict__ pos,
                                                  const float* __restrict__ nrm, uint32_t P, uint32_t spp,
                                                  rlc_samples in, float* __restrict__ radiance,
                                                  float* __restrict__ contrib, float* __restrict__ reward) {
    uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    size_t i = (size_t)b * kBlock + threadIdx.x;
    size_t n = (size_t)P * spp;
    bool valid = i < n;
    float e[3] = {0.0f, 0.0f, 0.0f};
    uint32_t p = 0, k = 0;
    if (valid) {
        p = (uint32_t)(i / spp);
        k = (uint32_t)(i % spp);
        float x[3] = {pos[3 * (size_t)p], pos[3 * (size_t)p + 1], pos[3 * (size_t)p + 2]};
        float nn[3] = {nrm[3 * (size_t)p], nrm[3 * (size_t)p + 1], nrm[3 * (size_t)p + 2]};
        float y[3] = {in.d_y[3 * i], in.d_y[3 * i + 1], in.d_y[3 * i + 2]};
        uint32_t l = in.d_light[i];
        float c[3];
        contribution(fp, x, nn, l, y, c);
        float ip = in.d_inv_pdf[i];
        e[0] = c[0] * ip;
        e[1] = c[1] * ip;
        e[2] = c[2] * ip;
        if (contrib) {
            contrib[3 * i] = c[0];
            contrib[3 * i + 1] = c[1];
            contrib[3 * i + 2] = c[2];
        }
        // cluster size for the reward: from the table the sample used
        uint32_t s = in.d_slot[i];
        uint32_t size = 1u;
        if (fp.reward_mode == 1u) {
            uint32_t cell = in.d_cell[i];
            const uint32_t* end = (cell != RLC_NONE && in.d_ready[i]) ? fp.cells.end + (size_t)cell * fp.cells.M
                                                                       : fp.tmpl.end;
            size = end[s] - (s ? end[s - 1u] : 0u);
        }
        float r = reward_of(fp, c, size);
        if (!(r <= 3.402823466e38f)) atomicOr(fp.err, RLC_DERR_NONFINITE);
        if (reward) reward[i] = r;
    }
    if (pow2_le64(spp)) {
        __shared__ float s_e[kBlock][3];
        point_sums(s_e, e, spp, valid, k, p, radiance);
    } else if (valid) {
        const float inv_spp = 1.0f / (float)spp;
        atomicAdd(&radiance[3 * (size_t)p], e[0] * inv_spp);
        atomicAdd(&radiance[3 * (size_t)p + 1], e[1] * inv_spp);
        atomicAdd(&radiance[3 * (size_t)p + 2], e[2] * inv_spp);
    }
}

__global__ void __launch_bounds__(kBlock) k_learn(FrameParams fp, rlc_samples in, const float* __restrict__ reward,
                                                  uint32_t n) {
    __shared__ AggTable agg;
    agg_clear(agg);
    __syncthreads();
    uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    size_t i = (size_t)b * kBlock + threadIdx.x;
    // draws of the learned proposal do not feed Eq. 1
    if (i < n && !(in.d_comp && in.d_comp[i]))
        agg_add(agg, fp, in.d_cell[i], in.d_slot[i], reward_fixed(fp, reward[i]));
    __syncthreads();
    agg_flush(agg, fp);
}

// The grid's pointers and t_lo for the shadow ray, as values defined just
// before it (an empty asm statement hides where they came from), so that
// their live range is the walk alone.  Short of SGPRs (the batch kernel
// holds its loop state besides), the compiler would otherwise park them in
// VGPR lanes and read each dword back, one VALU instruction apiece, at every
// step of the walk.  The casts keep the loads in the global address space.
__device__ __forceinline__ DevOcc walk_operands(const FrameParams& fp, float& t_lo) {
    typedef __attribute__((address_space(1))) const uint32_t* GU32;
    typedef __attribute__((address_space(1))) const float4* GF4;
    DevOcc occ = fp.occ;
    GU32 head = (GU32)occ.head;
    GU32 ref = (GU32)occ.ref;
    GF4 box = (GF4)occ.box;
    t_lo = fp.t_lo;
    asm volatile("" : "+s"(head), "+s"(ref), "+s"(box), "+s"(t_lo));
    occ.head = (const uint32_t*)head;
    occ.ref = (const uint32_t*)ref;
    occ.box = (const float4*)box;
    return occ;
}

// One block's samples i0 + threadIdx.x of a pass: sample, shade and learn
// (section 3).  Sample i belongs to point q = i / spp, sample k = i % spp;
// with a point order `perm` the point is perm[q] (its random numbers and
// radiance are those of that point, so any order gives the same results).
// The aggregation table must be clear on entry and is clear on exit; the
// block is synchronised on exit.
__device__ __forceinline__ void frame_block(const FrameParams& fp, const float* __restrict__ pos,
                                            const float* __restrict__ nrm, const uint32_t* __restrict__ perm,
                                            uint32_t P, uint32_t spp, uint32_t frame, float* __restrict__ radiance,
                                            size_t i0, AggTable& agg, float (*s_e)[3]) {
    const size_t i = i0 + threadIdx.x;
    const size_t n = (size_t)P * spp;
    const bool valid = i < n;
    float e[3] = {0.0f, 0.0f, 0.0f};
    uint32_t p = 0, k = 0;
    if (valid) {
        // a valid i is below P * spp < 2^32; spp is the same for every lane
        const uint32_t i32 = (uint32_t)i;
        uint32_t q = i32;
        if (spp != 1u) {
            q = i32 / spp;
            k = i32 - q * spp;
        }
        p = perm ? perm[q] : q;
        float x[3] = {pos[3 * (size_t)p], pos[3 * (size_t)p + 1], pos[3 * (size_t)p + 2]};
        float nn[3] = {nrm[3 * (size_t)p], nrm[3 * (size_t)p + 1], nrm[3 * (size_t)p + 2]};
        Sample sm;
        draw_sample(fp, x, nn, p, k, frame, sm);
        float c[3], d[3];
        if (contribution_unshadowed(fp, x, nn, sm.light, sm.y, c, d)) {
            float t_lo;
            const DevOcc occ = walk_operands(fp, t_lo);
            if (segment_blocked(occ, x, d, t_lo)) c[0] = c[1] = c[2] = 0.0f;
        }
        e[0] = c[0] * sm.inv_pdf;
        e[1] = c[1] * sm.inv_pdf;
        e[2] = c[2] * sm.inv_pdf;
        float r = reward_of(fp, c, sm.size);
        if (!(r <= 3.402823466e38f)) atomicOr(fp.err, RLC_DERR_NONFINITE);
        // only draws from the cell's own cut are uniform inside a cluster,
        // as Eq. 1's statistics assume
        if (!sm.comp) agg_add(agg, fp, sm.cell, sm.s, reward_fixed(fp, r));
        if (fp.log_node) {
            const size_t li = (size_t)p * spp + k;
            fp.log_pid[li] = p;
            fp.log_node[li] = sm.fnode;
            fp.log_w[li] = ((c[0] + c[1]) + c[2]) * sm.inv_pdf;
        }
    }
    __syncthreads();
    agg_flush(agg, fp);
    if (spp == 1u) {
        // one sample per point: its estimate is the point's sum (times 1/1)
        if (valid) {
            radiance[3 * (size_t)p] = e[0];
            radiance[3 * (size_t)p + 1] = e[1];
            radiance[3 * (size_t)p + 2] = e[2];
        }
    } else if (pow2_le64(spp)) {
        point_sums(s_e, e, spp, valid, k, p, radiance);
    } else if (valid) {
        const float inv_spp = 1.0f / (float)spp;
        atomicAdd(&radiance[3 * (size_t)p], e[0] * inv_spp);
        atomicAdd(&radiance[3 * (size_t)p + 1], e[1] * inv_spp);
        atomicAdd(&radiance[3 * (size_t)p + 2], e[2] * inv_spp);
    }
    __syncthreads();
}

// Sub-frame passes: acc = acc + x, and on the last pass (acc + x) * scale.
__global__ void __launch_bounds__(kBlock) k_accum(float* __restrict__ acc, const float* __restrict__ x, size_t n,
                                                  float scale, uint32_t finish) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float v = acc[i] + x[i];
    acc[i] = finish ? v * scale : v;
}

// Blocks dealt to the 8 XCDs in chunks of kXcdChunk neighbouring blocks,
// round robin: every XCD gets chunks from all over the image, so the cost of
// its walks follows the image's average, while the blocks it runs at a time
// still cover a few compact regions that share its L2.  The last,
// incomplete round is split into one contiguous range per XCD.
constexpr uint32_t kXcdChunk = 32;

__device__ __forceinline__ uint32_t xcd_chunk_block(uint32_t b, uint32_t nb) {
    const uint32_t round = 8u * kXcdChunk;
    const uint32_t full = (nb / round) * round;
    if (b >= full) return full + xcd_block(b - full, nb - full);
    const uint32_t x = b & 7u, j = b >> 3;
    return ((j / kXcdChunk) * 8u + x) * kXcdChunk + j % kXcdChunk;
}

// Fused pass: one lane per sample.  The parameters (the first argument,
// kept first) are read in place in the kernarg segment.  With an order, the
// launched blocks take the logical blocks longest first (the costliest
// blocks of the pass before start first, so that the pass does not end on a
// few of them running alone); each logical block records its duration.
__global__ void __launch_bounds__(kBlock, 8) k_frame(FrameParams /* read in place */, const float* __restrict__ pos,
                                                  const float* __restrict__ nrm, uint32_t P, uint32_t spp,
                                                  uint32_t frame, float* __restrict__ radiance) {
    __shared__ AggTable agg;
    __shared__ float s_e[kBlock][3];
    const FrameParams& fp = first_kernel_arg<FrameParams>();
    const unsigned long long t0 = wall_clock64();
    agg_clear(agg);
    __syncthreads();
    uint32_t b = xcd_chunk_block(blockIdx.x, gridDim.x);
    if (fp.blk_order) {
        const uint32_t o = fp.blk_order[blockIdx.x];
        b = o < gridDim.x ? o : b;
    }
    frame_block(fp, pos, nrm, nullptr, P, spp, frame, radiance, (size_t)b * kBlock, agg, s_e);
    if (fp.blk_cost && threadIdx.x == 0) {
        const unsigned long long d = wall_clock64() - t0;
        fp.blk_cost[b] = d < 0xFFFFFFFFull ? (uint32_t)d : 0xFFFFFFFFu;
    }
}

// Batched pass over several scenes: persistent blocks take work items of
// `rounds` x 256 samples, either from a counter (dynamic) or as contiguous
// ranges assigned per XCD (static).  Item -> scene by the scenes' first items.
__global__ void __launch_bounds__(kBlock, 7) k_batch_frame(const BatchScene* __restrict__ scenes, uint32_t n_scenes,
                                                        uint32_t total_items, uint32_t rounds, uint32_t dynamic,
                                                        uint32_t* __restrict__ counter,
                                                        const uint32_t* __restrict__ frame_ptr) {
    __shared__ AggTable agg;
    __shared__ float s_e[kBlock][3];
    __shared__ uint32_t s_item;
    agg_clear(agg);
    const uint32_t frame = *frame_ptr;
    const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t per_block = (total_items + gridDim.x - 1) / gridDim.x;
    uint32_t next = lb * per_block;
    const uint32_t stop = min(total_items, next + per_block);
    __syncthreads();
    for (;;) {
        uint32_t item;
        if (dynamic) {
            if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(s_item);
            if (item >= total_items) break;
        } else {
            if (next >= stop) break;
            item = next++;
        }
        uint32_t sc = 0;
        while (sc + 1u < n_scenes && scenes[sc + 1u].item_begin <= item) ++sc;
        // the scene's entry is the same for every lane (item and sc are)
        typedef const __attribute__((address_space(4))) FrameParams* ConstFrameParams;
        const FrameParams& fps = opaque_const((ConstFrameParams)uniform_u64((uint64_t)&scenes[sc].fp));
        const BatchScene& S = scenes[sc];
        const size_t first = (size_t)(item - S.item_begin) * rounds * kBlock;
        for (uint32_t r = 0; r < rounds; ++r)
            frame_block(fps, S.pos, S.nrm, S.perm, S.P, S.spp, frame, S.radiance, first + (size_t)r * kBlock, agg,
                        s_e);
    }
}

__global__ void k_batch_begin(uint32_t* counter) { *counter = 0u; }
__global__ void k_batch_end(uint32_t* frame) { *frame += 1u; }
__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

__global__ void __launch_bounds__(kBlock) k_cell_lin(FrameParams fp, const float* __restrict__ pos, uint32_t n,
                                                     uint32_t* __restrict__ lin, uint32_t* __restrict__ idx) {
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    lin[i] = cell_linear(fp, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]);
    idx[i] = (uint32_t)i;
}

__global__ void k_zero_f32(float* a, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.0f;
}

__global__ void __launch_bounds__(kBlock) k_cell_keys(FrameParams fp, const float* __restrict__ pos, uint32_t n,
                                                      uint64_t* __restrict__ keys) {
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    uint32_t lin = cell_linear(fp, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]);
    keys[i] = ((uint64_t)fp.scene_id << 32) | (uint64_t)lin;
}

inline uint32_t blocks_for(size_t n) { return (uint32_t)((n + kBlock - 1) / kBlock); }

hipError_t zero_radiance_if_needed(float* radiance, uint32_t P, uint32_t spp, hipStream_t s) {
    if (spp <= 64u && (spp & (spp - 1u)) == 0u) return hipSuccess;
    size_t n = (size_t)P * 3;
    hipLaunchKernelGGL(k_zero_f32, dim3(blocks_for(n)), dim3(kBlock), 0, s, radiance, n);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sample(const FrameParams& fp, const float* pos, const float* nrm, uint32_t P, uint32_t spp,
                         uint32_t frame, const rlc_samples& out, hipStream_t s) {
    size_t n = (size_t)P * spp;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sample, dim3(blocks_for(n)), dim3(kBlock), 0, s, fp, pos, nrm, P, spp, frame, out);
    return hipGetLastError();
}

hipError_t launch_shade(const FrameParams& fp, const float* pos, const float* nrm, uint32_t P, uint32_t spp,
                        const rlc_samples& in, float* radiance, float* contrib, float* reward, hipStream_t s) {
    size_t n = (size_t)P * spp;
    if (n == 0) return hipSuccess;
    hipError_t e = zero_radiance_if_needed(radiance, P, spp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_shade, dim3(blocks_for(n)), dim3(kBlock), 0, s, fp, pos, nrm, P, spp, in, radiance,
                       contrib, reward);
    return hipGetLastError();
}

hipError_t launch_learn(const FrameParams& fp, const rlc_samples& in, const float* reward, uint32_t n,
                        hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_learn, dim3(blocks_for(n)), dim3(kBlock), 0, s, fp, in, reward, n);
    return hipGetLastError();
}

hipError_t launch_accum(float* acc, const float* x, size_t n, float scale, bool finish, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_accum, dim3(blocks_for(n)), dim3(kBlock), 0, s, acc, x, n, scale, finish ? 1u : 0u);
    return hipGetLastError();
}

hipError_t launch_frame(const FrameParams& fp, const float* pos, const float* nrm, uint32_t P, uint32_t spp,
                        uint32_t frame, float* radiance, hipStream_t s) {
    size_t n = (size_t)P * spp;
    if (n == 0) return hipSuccess;
    hipError_t e = zero_radiance_if_needed(radiance, P, spp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_frame, dim3(blocks_for(n)), dim3(kBlock), 0, s, fp, pos, nrm, P, spp, frame, radiance);
    return hipGetLastError();
}

hipError_t launch_cell_keys(const FrameParams& fp, const float* pos, uint32_t n, uint64_t* keys, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_keys, dim3(blocks_for(n)), dim3(kBlock), 0, s, fp, pos, n, keys);
    return hipGetLastError();
}

hipError_t launch_cell_lin(const FrameParams& fp, const float* pos, uint32_t n, uint32_t* lin, uint32_t* idx,
                           hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_lin, dim3(blocks_for(n)), dim3(kBlock), 0, s, fp, pos, n, lin, idx);
    return hipGetLastError();
}

hipError_t launch_batch_begin(uint32_t* counter, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(1), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_batch_end(uint32_t* frame, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_end, dim3(1), dim3(1), 0, s, frame);
    return hipGetLastError();
}

hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_batch_frame(const BatchScene* scenes, uint32_t n_scenes, uint32_t total_items, uint32_t rounds,
                              uint32_t dynamic, uint32_t grid, uint32_t* counter, const uint32_t* frame,
                              hipStream_t s) {
    if (total_items == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_frame, dim3(grid), dim3(kBlock), 0, s, scenes, n_scenes, total_items, rounds, dynamic,
                       counter, frame);
    return hipGetLastError();
}

}  // namespace rlc
