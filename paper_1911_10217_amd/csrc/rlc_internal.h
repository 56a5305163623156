// Internal declarations of librlc: device-side views of the library's
// buffers, the per-sample device routines shared by the split and fused
// kernels, and the host launchers of every kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rlc.h"
#include "occ_trace.h"

#define RLC_NONE 0xFFFFFFFFu
#define RLC_EMPTY_KEY 0xFFFFFFFFFFFFFFFFull

// device error word bits
#define RLC_DERR_CAPACITY 1u
#define RLC_DERR_NONFINITE 2u
#define RLC_DERR_INPUT 4u
#define RLC_DERR_FX_OVERFLOW 8u   // a (cell, cluster) fixed-point reward sum wrapped 64 bits
#define RLC_DERR_WAIT 16u         // a lookup gave up waiting for another wave to publish a cell's row
#define RLC_HASH_MAX_PROBES 256u  // probes of the cell hash before a lookup reports the table full
#define RLC_MIX_M 64u           // nodes of the learned proposal's fixed cut (row stride of its cdf)
#define RLC_MAX_LEVELS 16u      // footprint-sized cells: levels of cell size

namespace rlc {

// Reference light tree in tree (Morton) order.  rec holds 64 bytes per light:
// {v0.xyz v1.x} {v1.yz v2.xy} {v2.z Le.rgb} {area normal.xyz}.
struct DevTree {
    const float4* rec;
    const uint32_t* left;
    const uint32_t* right;
    const uint32_t* parent;
    const uint32_t* first;
    const uint32_t* last;
    // per internal node i: (left, right, split, parent) with split the first
    // light of the right child, so one load gives all a split-collapse step
    // needs to know about a cut node
    const uint4* inode;
    uint32_t N;
};

// The initial cut: node ids, cluster ends, and the uniform Q~ / C a fresh
// cell samples with.
struct DevCut {
    const uint32_t* node;
    const uint32_t* end;
    const float* Qt;
    const float* C;
    uint32_t Meff;
};

// Cell tables.  A created cell's tables live in a row taken from a pool in
// creation order, so the rows in use are dense whatever the size of the
// lookup table; row r of every per-row array starts at r * M.  A lookup slot
// holds (row << 32) | the cell's linear index (RLC_EMPTY_KEY: free).  One
// context holds the cells of one scene, so the linear index is the key.
struct DevCells {
    unsigned long long* keys;   // per lookup slot
    uint32_t* ready;            // per row: 1 once the cell's own table exists
    uint32_t* node;
    uint32_t* end;
    float* Q;
    float* Qt;
    float* C;
    unsigned long long* sum;    // fixed-point reward sums of the pass
    uint32_t* cnt;              // sample counts of the pass
    uint32_t* live;             // per row: its lookup slot
    uint32_t* n_live;           // per stripe, RLC_NLIVE_STRIDE words apart: rows taken (passes stripe_rows once full)
    uint32_t capacity;          // lookup slots: dense, cells of the grid; hashed, 2^k
    uint32_t rows;              // rows in the pool
    uint32_t stripes;           // stripes of the pool, a power of two up to RLC_ROW_STRIPES_MAX
    uint32_t stripe_rows;       // rows per stripe: stripe s holds rows s, s + stripes, s + 2 stripes, ...
    uint32_t hashed;
    uint32_t M;                 // row stride
};
#define RLC_ROW_STRIPES_MAX 64u
// Words between two stripes' row counters: each counter in a 256-byte
// block of its own, so that the atomics of different stripes do not queue on
// one cache line.
#define RLC_NLIVE_STRIDE 64u

struct FrameParams {
    DevTree tree;
    DevCut tmpl;
    DevCells cells;
    DevOcc occ;
    float grid_lo[3];
    float inv_cell[3];
    uint32_t dims[3];
    uint32_t normal_bits;       // 2^normal_bits bins per octahedral normal coordinate
    float jitter;               // lookup jitter, in cells and normal bins
    float jit_reach[3];         // jitter x cell size, per axis
    uint32_t scene_id;
    uint32_t seed_lo, seed_hi;
    // footprint-sized cells: per point id the side of its footprint (null:
    // the finest level everywhere), the level count, the tile, the finest
    // cell edge, and the first linear index of every level
    const float* footprint;
    uint32_t fp_levels;
    float fp_tile;
    float fp_base;
    uint32_t lvl_first[RLC_MAX_LEVELS + 1];
    float f_r;
    float t_lo;
    float reward_max;
    float fx_scale;             // 2^fx_shift
    uint32_t reward_mode;
    uint32_t two_sided;
    uint32_t* err;
    // learned proposal: per-point inclusive running sums of the fixed cut's
    // probabilities (rows of RLC_MIX_M), or null for draws from the cut alone
    const float* mix_cdf;
    const uint32_t* fix_end;    // cluster ends of the fixed cut
    uint32_t fix_M;
    float mix_w;                // probability of drawing from the learned proposal
    // optional per-sample training records, index point * spp + sample
    uint32_t* log_pid;
    uint32_t* log_node;
    float* log_w;
    // block scheduling of the fused kernel (both optional): the logical
    // block each launched block runs (longest first, from the costs of the
    // pass before), and where each logical block records its duration
    const uint32_t* blk_order;
    uint32_t* blk_cost;
};

// Samples per block of the fused kernel, and the largest block count whose
// blocks are ordered longest first.
#define RLC_FRAME_BLOCK 256u
#define RLC_ORDER_MAX_BLOCKS 65536u

// One scene of a batched pass: its parameters, inputs and output, and the
// first work item that belongs to it.
struct BatchScene {
    FrameParams fp;
    const float* pos;
    const float* nrm;
    const uint32_t* perm;       // point visiting order, or null for input order
    float* radiance;
    uint32_t P;
    uint32_t spp;
    uint32_t item_begin;
    uint32_t items;
};

struct AdaptParams {
    DevTree tree;
    DevCut tmpl;
    DevCells cells;
    float alpha;
    float T;
    float eps;
    float fx_inv;               // 2^-fx_shift
    uint32_t adapt;
    uint32_t temporal;
    uint32_t split_steps;       // split-collapse steps per pass, at most (0 and 1: one)
    // with blk_n > 0, the end-of-pass launch also orders the fused kernel's
    // blk_n blocks for the next pass, longest first by blk_cost
    const uint32_t* blk_cost;
    uint32_t* blk_order;
    uint32_t blk_n;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32 multiplies
// with a word permutation; the key advances by the Weyl constants between
// rounds.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3,
                                                       uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32 x 32 -> 64 product in one instruction (v_mad_u64_u32)
        const unsigned long long p0 = 0xD2511F53ull * x0;
        const unsigned long long p1 = 0xCD9E8D57ull * x2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ float unit24(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

// floor-quantise one coordinate into [0, dims)
__device__ __forceinline__ uint32_t axis_cell(float p, float lo, float inv, uint32_t dims) {
    float f = floorf((p - lo) * inv);
    if (!(f >= 0.0f)) return 0u;
    if (f >= (float)dims) return dims - 1u;
    return (uint32_t)f;
}

// Position cell (the first three dimensions of the cell grid).
__device__ __forceinline__ uint32_t cell_linear(const FrameParams& fp, float x, float y, float z) {
    uint32_t ix = axis_cell(x, fp.grid_lo[0], fp.inv_cell[0], fp.dims[0]);
    uint32_t iy = axis_cell(y, fp.grid_lo[1], fp.inv_cell[1], fp.dims[1]);
    uint32_t iz = axis_cell(z, fp.grid_lo[2], fp.inv_cell[2], fp.dims[2]);
    return ix + fp.dims[0] * (iy + fp.dims[1] * iz);
}

// Octahedral map of a unit vector onto [0,1]^2 (Cigolle, Donow, Evangelakos,
// Mara, McGuire, Meyer, JCGT 3(2) 2014): project onto |x|+|y|+|z| = 1, and
// for z < 0 fold the lower half over the square's diagonals.
__device__ __forceinline__ void octahedral_uv(const float n[3], float& u, float& v) {
    const float s = (fabsf(n[0]) + fabsf(n[1])) + fabsf(n[2]);
    float px = n[0] / s;
    float py = n[1] / s;
    if (n[2] < 0.0f) {
        const float fx = (1.0f - fabsf(py)) * (px >= 0.0f ? 1.0f : -1.0f);
        const float fy = (1.0f - fabsf(px)) * (py >= 0.0f ? 1.0f : -1.0f);
        px = fx;
        py = fy;
    }
    u = px * 0.5f + 0.5f;
    v = py * 0.5f + 0.5f;
}

// Two unit tangents of the normal n (Duff, Burgess, Christensen, Hery,
// Kensler, Liani, Villemin, JCGT 6(1) 2017).
__device__ __forceinline__ void tangent_frame(const float n[3], float t[3], float b[3]) {
    const float sign = n[2] >= 0.0f ? 1.0f : -1.0f;
    const float a = -1.0f / (sign + n[2]);
    const float bb = n[0] * n[1] * a;
    t[0] = 1.0f + sign * n[0] * n[0] * a;
    t[1] = sign * bb;
    t[2] = -sign * n[0];
    b[0] = bb;
    b[1] = sign + n[1] * n[1] * a;
    b[2] = -n[1];
}

// Level of the point's position cells (section 3: cells sized from the
// footprint of the shading point): the smallest level whose edge, the
// finest edge doubled once per level, reaches tile x footprint.
__device__ __forceinline__ uint32_t point_level(const FrameParams& fp, uint32_t pid) {
    if (!fp.footprint) return 0u;
    const float want = fp.fp_tile * fp.footprint[pid];
    float edge = fp.fp_base;
    uint32_t L = 0;
    while (L + 1u < fp.fp_levels && edge < want) {
        edge = edge * 2.0f;
        ++L;
    }
    return L;
}

// The sample's cell in the 5-D grid of section 3 (three position and two
// normal dimensions): the position, moved by up to jitter/2 cells of its
// level in the tangent plane, and the octahedral normal coordinates, moved
// by up to jitter/2 bins (Philox tag 4 per sample), quantised by floor, the
// position index shifted right by the point's level.  The linear index is
// first(L) + ix + dx_L (iy + dy_L (iz + dz_L (qu + 2^b qv))); without
// footprints, normal bins and jitter it is the position cell.
__device__ __forceinline__ uint32_t cell_linear5(const FrameParams& fp, const float x[3], const float n[3],
                                                 uint32_t pid, uint32_t k, uint32_t frame) {
    const uint32_t L = point_level(fp, pid);
    if (L == 0u && fp.normal_bits == 0u && !(fp.jitter > 0.0f)) return cell_linear(fp, x[0], x[1], x[2]);
    const uint32_t nb = 1u << fp.normal_bits;
    float p[3] = {x[0], x[1], x[2]};
    float u = 0.0f, v = 0.0f;
    if (fp.normal_bits) octahedral_uv(n, u, v);
    if (fp.jitter > 0.0f) {
        uint32_t w0 = pid, w1 = k, w2 = frame, w3 = (fp.scene_id << 16) | 4u;
        philox4x32_10(w0, w1, w2, w3, fp.seed_lo, fp.seed_hi);
        const float xi0 = unit24(w0) - 0.5f, xi1 = unit24(w1) - 0.5f;
        float t[3], b[3];
        tangent_frame(n, t, b);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float reach = fp.jit_reach[a] * (float)(1u << L);
            p[a] = x[a] + reach * (xi0 * t[a] + xi1 * b[a]);
        }
        if (fp.normal_bits) {
            u = u + ((unit24(w2) - 0.5f) * fp.jitter) / (float)nb;
            v = v + ((unit24(w3) - 0.5f) * fp.jitter) / (float)nb;
        }
    }
    const uint32_t ix = axis_cell(p[0], fp.grid_lo[0], fp.inv_cell[0], fp.dims[0]) >> L;
    const uint32_t iy = axis_cell(p[1], fp.grid_lo[1], fp.inv_cell[1], fp.dims[1]) >> L;
    const uint32_t iz = axis_cell(p[2], fp.grid_lo[2], fp.inv_cell[2], fp.dims[2]) >> L;
    const uint32_t qu = axis_cell(u, 0.0f, (float)nb, nb);
    const uint32_t qv = axis_cell(v, 0.0f, (float)nb, nb);
    const uint32_t dx = ((fp.dims[0] - 1u) >> L) + 1u;
    const uint32_t dy = ((fp.dims[1] - 1u) >> L) + 1u;
    const uint32_t dz = ((fp.dims[2] - 1u) >> L) + 1u;
    return fp.lvl_first[L] + (ix + dx * (iy + dy * (iz + dz * (qu + nb * qv))));
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
    // SplitMix64 finaliser (Steele, Lea, Flood 2014)
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    x ^= x >> 31;
    return x;
}

// Row field of a lookup slot while its cell is being created, and once the
// row pool turned out to be full.
#define RLC_ROW_PENDING 0xFFFFFFFEu
#define RLC_ROW_FULL 0xFFFFFFFDu
// polls of a pending slot before a lookup gives up (the creating wave
// publishes the row a few instructions after taking the slot)
#define RLC_CREATE_MAX_POLLS (1u << 16)

__device__ __forceinline__ uint32_t slot_row(unsigned long long w) { return (uint32_t)(w >> 32); }
__device__ __forceinline__ unsigned long long slot_word(uint32_t row, uint32_t lin) {
    return ((unsigned long long)row << 32) | (unsigned long long)lin;
}

// The row of slot h, whose word w holds this lookup's cell: waits while
// another wave publishes the row.  RLC_NONE (and an error bit) when the pool
// was full or the wait ran out.
__device__ __forceinline__ uint32_t resolve_row(const DevCells& c, uint32_t h, unsigned long long w, uint32_t* err) {
    uint32_t r = slot_row(w);
    for (uint32_t n = 0; r == RLC_ROW_PENDING && n < RLC_CREATE_MAX_POLLS; ++n) {
        __builtin_amdgcn_s_sleep(1);
        w = __hip_atomic_load(&c.keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        r = slot_row(w);
    }
    if (r == RLC_ROW_PENDING) {
        atomicOr(err, RLC_DERR_WAIT);
        return RLC_NONE;
    }
    if (r == RLC_ROW_FULL) {
        atomicOr(err, RLC_DERR_CAPACITY);
        return RLC_NONE;
    }
    return r;
}

// Create the cell with linear index lin at slot h, read as free, for the
// lanes of the wave that call this together (divergent code).  Lanes with
// the same key have probed the same slots, so they are here at the same
// slot, and one of them (the group's leader) acts for all: it claims the slot
// by compare-and-swap to (pending, lin), takes the next row of the slot's
// stripe of the pool and publishes (row, lin).  A slot meanwhile claimed by
// another wave for the same cell gives its row once published; one claimed
// for another cell sets `retry` (probe on).  Rows are taken only by
// successful claims, so the rows in use are each stripe's first
// min(n_live[s], stripe_rows).  The stripes (chosen by slot) each have their
// own counter, so the creations of a pass do not all queue on one atomic,
// and are interleaved row by row, so the rows in use stay packed at the
// start of the pool.
// Groups are served one after the other, so no lane waits on a claim of its
// own wave.
__device__ __forceinline__ uint32_t create_at(const DevCells& c, uint32_t h, uint32_t lin, uint32_t* err,
                                              bool& retry) {
    const uint32_t lane = __lane_id();
    unsigned long long pending = __ballot(1);
    uint32_t res = RLC_NONE;
    bool done = false;
    retry = false;
    while (pending) {
        const uint32_t leader = (uint32_t)__ffsll((long long)pending) - 1u;
        const uint32_t llin = (uint32_t)__builtin_amdgcn_readlane((int)lin, (int)leader);
        const bool mine = !done && lin == llin;
        pending &= ~__ballot(mine);
        uint32_t r = RLC_NONE, st = 0u;  // st: 0 answered, 1 the slot holds another cell
        if (lane == leader) {
            const unsigned long long old = atomicCAS(&c.keys[h], RLC_EMPTY_KEY, slot_word(RLC_ROW_PENDING, lin));
            if (old == RLC_EMPTY_KEY) {
                const uint32_t st = h & (c.stripes - 1u);
                const uint32_t k = atomicAdd(&c.n_live[st * RLC_NLIVE_STRIDE], 1u);
                if (k < c.stripe_rows) {
                    r = k * c.stripes + st;
                    c.live[r] = h;
                } else {
                    atomicOr(err, RLC_DERR_CAPACITY);
                    r = RLC_NONE;
                }
                atomicExch(&c.keys[h], slot_word(r == RLC_NONE ? RLC_ROW_FULL : r, lin));
            } else if ((uint32_t)old == lin) {
                r = resolve_row(c, h, old, err);
            } else {
                st = 1u;
            }
        }
        r = (uint32_t)__builtin_amdgcn_readlane((int)r, (int)leader);
        st = (uint32_t)__builtin_amdgcn_readlane((int)st, (int)leader);
        if (mine) {
            res = r;
            retry = st == 1u;
            done = true;
        }
    }
    return res;
}

// The row of a cell key, creating the cell if it is absent (RLC_NONE and the
// capacity error when the row pool is full or, hashed, when
// RLC_HASH_MAX_PROBES slots in a row hold other keys).  Creation only takes
// the row and records its slot in the live list; the cell's own table is
// filled at the end of the pass.  A slot changes from free to (pending, key)
// by compare-and-swap and then once more to (row, key), so the probe reads
// it with a plain (cached) load: a stale "free" only sends the lanes to the
// compare-and-swap and a stale "pending" to the coherent polls, which both
// see the current word.
__device__ __forceinline__ uint32_t find_or_create(const DevCells& c, unsigned long long key, uint32_t lin,
                                                   uint32_t* err) {
    if (!c.hashed) {
        if (lin >= c.capacity) return RLC_NONE;
        const unsigned long long w = c.keys[lin];
        if (w == RLC_EMPTY_KEY) {
            bool retry;
            return create_at(c, lin, lin, err, retry);
        }
        return slot_row(w) < c.rows ? slot_row(w) : resolve_row(c, lin, w, err);
    }
    uint32_t mask = c.capacity - 1u;
    uint32_t h = (uint32_t)mix64(key) & mask;
    // a lookup gives up after a bounded run of occupied slots, so a nearly
    // full table reports itself instead of walking all of its slots
    const uint32_t probes = c.capacity < RLC_HASH_MAX_PROBES ? c.capacity : RLC_HASH_MAX_PROBES;
    for (uint32_t probe = 0; probe < probes; ++probe) {
        const unsigned long long w = c.keys[h];
        if (w == RLC_EMPTY_KEY) {
            bool retry;
            const uint32_t r = create_at(c, h, lin, err, retry);
            if (!retry) return r;
        } else if ((uint32_t)w == lin) {
            return slot_row(w) < c.rows ? slot_row(w) : resolve_row(c, h, w, err);
        }
        h = (h + 1u) & mask;
    }
    atomicOr(err, RLC_DERR_CAPACITY);
    return RLC_NONE;
}

// ---------------------------------------------------------------------------
struct Sample {
    uint32_t cell;      // table row or RLC_NONE
    uint32_t ready;
    uint32_t comp;      // 1: drawn by the learned proposal
    uint32_t fnode;     // fixed-cut node holding the light (RLC_NONE if not needed)
    uint32_t s;
    uint32_t size;
    uint32_t light;
    float inv_pdf;
    float y[3];
    unsigned long long key;
};

__device__ __forceinline__ void draw_sample(const FrameParams& fp, const float xp[3], const float nrm[3], uint32_t pid,
                                            uint32_t k, uint32_t frame, Sample& o) {
    uint32_t lin = cell_linear5(fp, xp, nrm, pid, k, frame);
    unsigned long long key = ((unsigned long long)fp.scene_id << 32) | (unsigned long long)lin;
    uint32_t cell = find_or_create(fp.cells, key, lin, fp.err);
    uint32_t rdy = (cell != RLC_NONE) ? fp.cells.ready[cell] : 0u;
    const float* C;
    const float* Qt;
    const uint32_t* end;
    if (rdy) {
        size_t base = (size_t)cell * fp.cells.M;
        C = fp.cells.C + base;
        Qt = fp.cells.Qt + base;
        end = fp.cells.end + base;
    } else {
        C = fp.tmpl.C;
        Qt = fp.tmpl.Qt;
        end = fp.tmpl.end;
    }
    const uint32_t Meff = fp.tmpl.Meff;
    uint32_t w0 = pid, w1 = k, w2 = frame, w3 = fp.scene_id << 16;
    philox4x32_10(w0, w1, w2, w3, fp.seed_lo, fp.seed_hi);
    float u0 = unit24(w0);
    unsigned long long draw40 = ((unsigned long long)(w0 & 0xFFu) << 32) | (unsigned long long)w1;
    float u2 = unit24(w2);
    float u3 = unit24(w3);

    // mixture component: counter tag 1, only with the learned proposal on
    const float* q = nullptr;
    bool use_mlp = false;
    if (fp.mix_cdf) {
        uint32_t c0 = pid, c1 = k, c2 = frame, c3 = (fp.scene_id << 16) | 1u;
        philox4x32_10(c0, c1, c2, c3, fp.seed_lo, fp.seed_hi);
        q = fp.mix_cdf + (size_t)pid * RLC_MIX_M;
        use_mlp = unit24(c0) < fp.mix_w;
    }
    const float total = C[Meff - 1u];
    const uint32_t Mf = fp.fix_M;
    uint32_t s, l, kf = RLC_NONE, fsize = 0;
    if (!use_mlp) {
        // smallest s with t < C[s] (C is non-decreasing)
        float t = u0 * total;
        uint32_t lo = 0, hi = Meff;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (t < C[mid])
                hi = mid;
            else
                lo = mid + 1u;
        }
        s = lo < Meff ? lo : Meff - 1u;
        uint32_t b = s ? end[s - 1u] : 0u;
        l = b + (uint32_t)((draw40 * (unsigned long long)(end[s] - b)) >> 40);
    } else {
        // node of the fixed cut from the learned cdf, a light inside it, and
        // the cell's cluster that holds that light
        float t = u0 * q[Mf - 1u];
        uint32_t lo = 0, hi = Mf;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (t < q[mid])
                hi = mid;
            else
                lo = mid + 1u;
        }
        kf = lo < Mf ? lo : Mf - 1u;
        uint32_t fb = kf ? fp.fix_end[kf - 1u] : 0u;
        fsize = fp.fix_end[kf] - fb;
        l = fb + (uint32_t)((draw40 * (unsigned long long)fsize) >> 40);
        lo = 0;
        hi = Meff - 1u;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (l < end[mid])
                hi = mid;
            else
                lo = mid + 1u;
        }
        s = lo;
    }
    if (kf == RLC_NONE && (q || fp.log_node)) {
        uint32_t lo = 0, hi = Mf - 1u;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (l < fp.fix_end[mid])
                hi = mid;
            else
                lo = mid + 1u;
        }
        kf = lo;
        fsize = fp.fix_end[kf] - (kf ? fp.fix_end[kf - 1u] : 0u);
    }
    const uint32_t begin = s ? end[s - 1u] : 0u;
    const uint32_t size = end[s] - begin;
    float inv_pdf;
    if (q) {
        // p(l) = (1 - w) p_cut(l) + w p_learned(l), each uniform inside its
        // cluster or node
        float pt = Qt[s] / ((float)size * total);
        float qk = q[kf] - (kf ? q[kf - 1u] : 0.0f);
        float pm = qk / ((float)fsize * q[Mf - 1u]);
        inv_pdf = 1.0f / ((1.0f - fp.mix_w) * pt + fp.mix_w * pm);
    } else {
        inv_pdf = ((float)size * total) / Qt[s];
    }

    const float4 r0 = fp.tree.rec[4u * l + 0u];
    const float4 r1 = fp.tree.rec[4u * l + 1u];
    const float4 r2 = fp.tree.rec[4u * l + 2u];
    float su = sqrtf(u2);
    float b0 = 1.0f - su;
    float b1 = u3 * su;
    float b2 = (1.0f - b0) - b1;
    o.y[0] = (b0 * r0.x + b1 * r0.w) + b2 * r1.z;
    o.y[1] = (b0 * r0.y + b1 * r1.x) + b2 * r1.w;
    o.y[2] = (b0 * r0.z + b1 * r1.y) + b2 * r2.x;
    o.cell = cell;
    o.ready = rdy;
    o.comp = use_mlp ? 1u : 0u;
    o.fnode = kf;
    o.s = s;
    o.size = size;
    o.light = l;
    o.inv_pdf = inv_pdf;
    o.key = key;
}

// The unshadowed contribution Le f_r G A of the sampled point y as seen from
// x, and the segment d = y - x.  Returns false (cu = 0) when the sample
// cannot contribute whatever the visibility.
__device__ __forceinline__ bool contribution_unshadowed(const FrameParams& fp, const float x[3], const float n[3],
                                                       uint32_t l, const float y[3], float cu[3], float d[3]) {
    cu[0] = cu[1] = cu[2] = 0.0f;
    const float4 r2 = fp.tree.rec[4u * l + 2u];
    const float4 r3 = fp.tree.rec[4u * l + 3u];
    d[0] = y[0] - x[0];
    d[1] = y[1] - x[1];
    d[2] = y[2] - x[2];
    float dist2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    float area = r3.x;
    if (!(dist2 > 0.0f && area > 0.0f)) return false;
    float dist = sqrtf(dist2);
    float cos_x = ((n[0] * d[0] + n[1] * d[1]) + n[2] * d[2]) / dist;
    float dl = (r3.y * d[0] + r3.z * d[1]) + r3.w * d[2];
    float cos_l;
    if (fp.two_sided)
        cos_l = fabsf(dl) / dist;
    else
        cos_l = (dl < 0.0f ? -dl : 0.0f) / dist;
    if (!(cos_x > 0.0f && cos_l > 0.0f)) return false;
    float G = (cos_x * cos_l) / dist2;
    float kk = (fp.f_r * G) * area;
    if (!(kk > 0.0f && (r2.y > 0.0f || r2.z > 0.0f || r2.w > 0.0f))) return false;
    cu[0] = r2.y * kk;
    cu[1] = r2.z * kk;
    cu[2] = r2.w * kk;
    return true;
}

// Contribution c_l = Le f_r G A V of the sampled point y as seen from x.
__device__ __forceinline__ void contribution(const FrameParams& fp, const float x[3], const float n[3],
                                             uint32_t l, const float y[3], float c[3]) {
    float d[3];
    if (contribution_unshadowed(fp, x, n, l, y, c, d) && segment_blocked(fp.occ, x, d, fp.t_lo))
        c[0] = c[1] = c[2] = 0.0f;
}

__device__ __forceinline__ float reward_of(const FrameParams& fp, const float c[3], uint32_t size) {
    float r = (c[0] + c[1]) + c[2];
    if (fp.reward_mode == 1u) r = r * (float)size;
    return r;
}

__device__ __forceinline__ unsigned long long reward_fixed(const FrameParams& fp, float r) {
    float rc = r < fp.reward_max ? r : fp.reward_max;
    return (unsigned long long)rintf(rc * fp.fx_scale);
}

// sum += v on a fixed-point reward sum, latching the overflow error when
// the 64-bit sum wraps (old + v < old); the statistics are then not used.
__device__ __forceinline__ void add_fixed(unsigned long long* sum, unsigned long long v, uint32_t* err) {
    const unsigned long long old = atomicAdd(sum, v);
    if (old + v < old) atomicOr(err, RLC_DERR_FX_OVERFLOW);
}

// Parameters that stay the same for a whole launch, read through a pointer
// that an empty asm statement makes opaque, typed in the constant address
// space: each field is then loaded with s_load where it is used.  Read from
// a by-value kernel argument, the compiler loads the fields at the kernel's
// start and, short of SGPRs, keeps them in VGPR lanes and reads each dword
// back with a v_readlane (a VALU instruction), also inside loops.  The
// pointer must be the same for every lane of the wave.
template <class T>
__device__ __forceinline__ const T& opaque_const(const __attribute__((address_space(4))) T* p) {
    asm volatile("" : "+s"(p));
    return *(const T*)p;
}

// A kernel's first argument, of type T and passed by value, read in place at
// offset 0 of the kernarg segment (taking the argument's address would make
// a private copy of it).
template <class T>
__device__ __forceinline__ const T& first_kernel_arg() {
    return opaque_const((const __attribute__((address_space(4))) T*)__builtin_amdgcn_kernarg_segment_ptr());
}

// A 64-bit value that every lane holds, as the first lane's.  The builtin
// returns int: each half is taken as uint32_t before it is widened, so the
// low half is not sign-extended into the high one.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}

// Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous
// range of logical blocks so neighbouring points share one L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
    uint32_t q = nb >> 3, r = nb & 7u;
    uint32_t x = b & 7u, j = b >> 3;
    return x * q + (x < r ? x : r) + j;
}

}  // namespace rlc

// ---------------------------------------------------------------------------
// Host launchers (all enqueue on `s`; return hipError_t of the launch)
// ---------------------------------------------------------------------------
namespace rlc {
// tree.hip
hipError_t launch_tri_prep(const float* tri, uint32_t N, float* sums, float* part_lo, float* part_hi,
                           uint32_t nblocks, uint32_t* err, hipStream_t s);
hipError_t launch_bbox_final(const float* part_lo, const float* part_hi, uint32_t nparts, float* bbox,
                             hipStream_t s);
hipError_t launch_morton(const float* sums, const float* bbox, uint32_t N, uint32_t* keys, uint32_t* vals,
                         hipStream_t s);
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp,
                            uint32_t* hist, uint32_t N, int bits, hipStream_t s);
// Entries of the hist buffer radix_sort_pairs needs (histogram and scan scratch).
size_t radix_sort_hist_entries(uint32_t N);
// Exclusive scan in place; scratch: scan_scratch_entries(n) words.
size_t scan_scratch_entries(size_t n);
hipError_t launch_exclusive_scan(uint32_t* data, uint32_t n, uint32_t* scratch, hipStream_t s);
hipError_t launch_gather_records(const float* tri, const float* emit, const uint32_t* perm, uint32_t N,
                                 float4* rec, hipStream_t s);
hipError_t launch_invert_perm(const uint32_t* perm, uint32_t N, uint32_t* rank, hipStream_t s);
hipError_t launch_scatter_emission(const float* emit, const uint32_t* rank, uint32_t N, float4* rec,
                                   hipStream_t s);
hipError_t launch_radix_tree(const uint32_t* morton, const uint32_t* perm, uint32_t N, uint32_t* left,
                             uint32_t* right, uint32_t* parent, uint32_t* first, uint32_t* last, uint32_t* inode,
                             hipStream_t s);
hipError_t launch_initial_cut(DevTree tree, uint32_t M, uint32_t* node, uint32_t* end, float* Qt, float* C,
                              hipStream_t s);
hipError_t launch_check_finite(const float* a, uint32_t n, uint32_t* err, hipStream_t s);
// Latches RLC_DERR_INPUT for a negative or non-finite entry.
hipError_t launch_check_nonneg(const float* a, uint32_t n, uint32_t* err, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* a, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* a, unsigned long long v, size_t n, hipStream_t s);

// occ.hip
hipError_t launch_pack_boxes(const float* aabb, uint32_t K, float4* box, float* part_lo, float* part_hi,
                             uint32_t nblocks, uint32_t* err, hipStream_t s);
hipError_t launch_occ_count(const float4* box, uint32_t K, DevOcc occ, uint32_t* counts, hipStream_t s);
hipError_t launch_occ_sizes(const uint32_t* counts, uint32_t ncell, uint32_t* sizes, hipStream_t s);
hipError_t launch_occ_lists(const float4* box, uint32_t K, DevOcc occ, const uint32_t* counts, uint32_t* start,
                            uint32_t* cursor, uint32_t* head, uint32_t* ref, hipStream_t s);
// Writes the eight octant radii into the header of every cell no box
// overlaps (tmp0, tmp1: res^3 words each).
hipError_t launch_occ_skip(uint32_t* head, uint32_t* tmp0, uint32_t* tmp1, uint32_t res, hipStream_t s);
hipError_t launch_visible(DevOcc occ, float t_lo, const float* x, const float* y, uint32_t n, uint8_t* vis,
                          hipStream_t s);

// frame.hip
hipError_t launch_sample(const FrameParams& fp, const float* pos, const float* nrm, uint32_t P, uint32_t spp,
                         uint32_t frame, const rlc_samples& out, hipStream_t s);
hipError_t launch_shade(const FrameParams& fp, const float* pos, const float* nrm, uint32_t P, uint32_t spp,
                        const rlc_samples& in, float* radiance, float* contrib, float* reward, hipStream_t s);
hipError_t launch_learn(const FrameParams& fp, const rlc_samples& in, const float* reward, uint32_t n,
                        hipStream_t s);
// acc[i] = acc[i] + x[i] over n floats; with finish, then times scale.
hipError_t launch_accum(float* acc, const float* x, size_t n, float scale, bool finish, hipStream_t s);
hipError_t launch_frame(const FrameParams& fp, const float* pos, const float* nrm, uint32_t P, uint32_t spp,
                        uint32_t frame, float* radiance, hipStream_t s);
hipError_t launch_cell_keys(const FrameParams& fp, const float* pos, uint32_t n, uint64_t* keys, hipStream_t s);
hipError_t launch_cell_lin(const FrameParams& fp, const float* pos, uint32_t n, uint32_t* lin, uint32_t* idx,
                           hipStream_t s);
hipError_t launch_batch_begin(uint32_t* counter, hipStream_t s);
hipError_t launch_batch_end(uint32_t* frame, hipStream_t s);
hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s);
hipError_t launch_batch_frame(const BatchScene* scenes, uint32_t n_scenes, uint32_t total_items, uint32_t rounds,
                              uint32_t dynamic, uint32_t grid, uint32_t* counter, const uint32_t* frame,
                              hipStream_t s);

// adapt.hip
hipError_t launch_adapt(const AdaptParams& ap, hipStream_t s);
// Meff: the largest cut size of the batch's scenes.
hipError_t launch_batch_adapt(const AdaptParams* aps, uint32_t n_scenes, uint32_t Meff, hipStream_t s);
// The batch's cells with cuts of up to 64 clusters and one split-collapse
// step, 16 cells per block over all scenes' rows in use (1 to 16 scenes).
hipError_t launch_batch_adapt16(const AdaptParams* aps, uint32_t n_scenes, hipStream_t s);
// Checkpoint load of n cells (keys, cuts and Q of Meff entries each).
hipError_t launch_load_cells(const AdaptParams& ap, const unsigned long long* keys, const uint32_t* node,
                             const float* Q, uint32_t n, uint32_t* err, hipStream_t s);
hipError_t launch_gather_cells(DevCells c, uint32_t Meff, const uint32_t* rows, uint32_t n, uint32_t* node,
                               uint32_t* end, float* Q, float* Qt, float* C, unsigned long long* sum,
                               uint32_t* cnt, hipStream_t s);

// stats.hip
hipError_t launch_image_error(const float* img, const float* ref, uint32_t n, double* partial,
                              uint32_t nblocks, hipStream_t s);
}  // namespace rlc
