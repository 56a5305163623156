// End-of-pass adaptation of every cell that received samples (section 3):
// Eq. 1 over the pass in its batch form, one split-collapse step, Q~ and the
// cdf C by Eq. 2.  One wavefront per cell; slot s of the cut lives in lane
// s % 64 (up to four slots per lane for cuts of up to 256 clusters).
#include "rlc_internal.h"

namespace rlc {

namespace {

constexpr int kWave = 64;
constexpr int kMaxPerLane = RLC_MMAX / kWave;
static_assert(kMaxPerLane == 4, "k_adapt instances cover one and four slots per lane");

__device__ __forceinline__ float pow_uint(float a, uint32_t n) {
    float res = 1.0f, b = a;
    while (n) {
        if (n & 1u) res = res * b;
        b = b * b;
        n >>= 1;
    }
    return res;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, kWave);
        v = o < v ? o : v;
    }
    return v;
}

// Per-cell scratch in LDS, S = 64 PER entries per array: the cut's nodes,
// ends (one past the cluster's last light), the cluster nodes' parents, Q,
// the new cut's nodes and parents, and two arrays that hold the new cut's
// ends and Q during split-collapse, then Q~ and C.
struct AdaptLds {
    uint32_t* node;
    uint32_t* end;
    uint32_t* par;
    float* Q;
    uint32_t* nnode;
    uint32_t* npar;
    uint32_t* nend;
    float* Qt;  // aliases nend
    float* nQ;
    float* C;   // aliases nQ
};

constexpr uint32_t kLdsArrays = 8;

__device__ __forceinline__ AdaptLds lds_view(uint32_t* base, uint32_t S) {
    AdaptLds L;
    L.node = base;
    L.end = base + S;
    L.par = base + 2 * S;
    L.Q = reinterpret_cast<float*>(base + 3 * S);
    L.nnode = base + 4 * S;
    L.nend = base + 5 * S;
    L.Qt = reinterpret_cast<float*>(base + 5 * S);
    L.nQ = reinterpret_cast<float*>(base + 6 * S);
    L.C = reinterpret_cast<float*>(base + 6 * S);
    L.npar = base + 7 * S;
    return L;
}

// Lane s's value of v, read by a whole-wave (uniform) index s.
__device__ __forceinline__ float lane_value(float v, uint32_t s) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), (int)s));
}

// Orders one wavefront's LDS accesses (the cell's scratch is the wave's
// own, so no other wave takes part).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The floor eps S / Meff of Eq. 2.  With eps > 0 it never underflows to 0
// (Q decays towards subnormals in cells whose rewards stay 0): at least the
// smallest normal float, so every cluster keeps p > 0.
__device__ __forceinline__ float eq2_floor(const AdaptParams& ap, float S, uint32_t Meff) {
    float fl = (ap.eps * S) / (float)Meff;
    if (ap.eps > 0.0f && fl < 1.17549435e-38f) fl = 1.17549435e-38f;
    return fl;
}

// What a cell's end of pass reads from the tables before it starts: its
// counts, ready flag, stored cut and Q, reward sums, and the initial cut's
// entries (for a fresh cell).  Loaded for every slot without waiting on the
// flag, so all of it is one round of independent loads that can be issued
// while the wave still works on the previous cell; a fresh cell's stored
// row is read but not used.
template <int PER>
struct CellIn {
    uint32_t c, ready;
    uint32_t cnt[PER], node[PER], end[PER], tnode[PER], tend[PER];
    float q[PER];
    unsigned long long sum[PER];
    // each slot's node record (children, split point, parent; a leaf: its
    // parent alone), by load_cell_nodes
    uint4 nrec[PER];
};

template <int PER>
__device__ __forceinline__ void load_cell(const AdaptParams& ap, uint32_t c, CellIn<PER>& in) {
    const DevCells& cells = ap.cells;
    const uint32_t Meff = ap.tmpl.Meff;
    const size_t base = (size_t)c * cells.M;
    in.c = c;
    in.ready = cells.ready[c];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint32_t s = (threadIdx.x & (kWave - 1u)) + kWave * j;
        const bool ok = s < Meff;
        const size_t i = base + (ok ? s : 0u);
        const uint32_t st = ok ? s : 0u;
        in.cnt[j] = ok ? cells.cnt[i] : 0u;
        in.node[j] = cells.node[i];
        in.end[j] = cells.end[i];
        in.q[j] = cells.Q[i];
        in.sum[j] = cells.sum[i];
        in.tnode[j] = ap.tmpl.node[st];
        in.tend[j] = ap.tmpl.end[st];
    }
}

// The node record of each slot's cluster, for the cut the pass starts from
// (the stored one, or the initial cut for a fresh cell).  Issued once the
// cell's row has arrived, ahead of the cell's work.  A node outside the tree
// (only in a row that is not in use) reads nothing.
template <int PER>
__device__ __forceinline__ void load_cell_nodes(const AdaptParams& ap, CellIn<PER>& in) {
    const uint32_t Meff = ap.tmpl.Meff;
    const bool fresh = in.ready == 0u || ap.temporal == 0u;
    const uint32_t n_nodes = 2u * ap.tree.N - 1u;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint32_t s = (threadIdx.x & (kWave - 1u)) + kWave * j;
        in.nrec[j] = make_uint4(0u, 0u, 0u, RLC_NONE);
        if (s < Meff) {
            const uint32_t nd = fresh ? in.tnode[j] : in.node[j];
            if (nd + 1u < ap.tree.N)
                in.nrec[j] = ap.tree.inode[nd];
            else if (nd < n_nodes)
                in.nrec[j].w = ap.tree.parent[nd];
        }
    }
}

// End of pass for the cell loaded into in, by one wavefront, in the wave's
// own LDS scratch L; PER slots per lane (cuts of up to 64 PER clusters).
// The front: Eq. 1 and split-collapse, leaving the new cut and Q in L.
// Returns false (and does nothing) when the cell had no samples this pass.
template <int PER>
__device__ __forceinline__ bool adapt_front(const AdaptParams& ap, const CellIn<PER>& in, const AdaptLds& L) {
    const DevCells& cells = ap.cells;
    const uint32_t lane = threadIdx.x & (kWave - 1u);
    const uint32_t Meff = ap.tmpl.Meff;
    const uint32_t c = in.c;
    const size_t base = (size_t)c * cells.M;
    bool any = false;
#pragma unroll
    for (int j = 0; j < PER; ++j) any |= in.cnt[j] != 0u;
    if (!__any(any)) return false;  // no samples this pass: the cell is left as it is

    const bool fresh = in.ready == 0u || ap.temporal == 0u;
    // the children and split point of each cluster's node, for the first
    // step's split (they come with the parent in one load)
    uint32_t pre_l[PER], pre_r[PER], pre_sp[PER];
    // the cut and Q (a fresh cell starts from the initial cut, Q = 0)
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        uint32_t s = lane + kWave * j;
        pre_l[j] = pre_r[j] = pre_sp[j] = 0u;
        if (s < Meff) {
            const uint32_t nd = fresh ? in.tnode[j] : in.node[j];
            const uint32_t en = fresh ? in.tend[j] : in.end[j];
            float q = fresh ? 0.0f : in.q[j];
            // the tree lookup the step needs for every cluster: its parent,
            // and for an internal node its children and split point
            pre_l[j] = in.nrec[j].x;
            pre_r[j] = in.nrec[j].y;
            pre_sp[j] = in.nrec[j].z;
            L.par[s] = in.nrec[j].w;
            L.end[s] = en;
            if (ap.temporal && in.cnt[j]) {
                // Eq. 1 applied to the n samples of the pass at once
                float a_n = pow_uint(1.0f - ap.alpha, in.cnt[j]);
                float m = ((float)in.sum[j] * ap.fx_inv) / (float)in.cnt[j];
                float t1 = a_n * q;
                float t2 = (1.0f - a_n) * m;
                q = t1 + t2;
            }
            L.node[s] = nd;
            L.Q[s] = q;
        }
    }
    wave_sync();

    // ---- split-collapse: steps until one changes nothing, at most
    // max(split_steps, 1) of them (one step: the basic algorithm) ----
    if (ap.temporal && ap.adapt && Meff >= 2u) {
        const uint32_t steps = ap.split_steps > 1u ? ap.split_steps : 1u;
        for (uint32_t step = 0; step < steps; ++step) {
            // after this step another may follow: keep the parents current
            const bool more = step + 1u < steps;
            bool changed = false;
            uint32_t smax = RLC_NONE, smin = RLC_NONE;
            float qpmin = 0.0f;
            if constexpr (PER == 1) {
                // one slot per lane, slot = lane: a 32-bit wave maximum (minimum)
                // of the Q bits (Q >= 0, so their order as integers is the
                // floats' order), then the lowest lane holding it
                const uint32_t s = lane;
                const bool split_ok = s < Meff && L.end[s] - (s ? L.end[s - 1u] : 0u) > 1u;
                const uint32_t qbits = split_ok ? __float_as_uint(L.Q[s]) : 0u;
                const uint32_t qmax = __reduce_max_sync(~0ull, qbits);
                const unsigned long long at_max = __ballot(split_ok && qbits == qmax);
                if (at_max) smax = (uint32_t)__ffsll((long long)at_max) - 1u;
                bool pair_ok = false;
                uint32_t pbits = 0xFFFFFFFFu;
                if (s + 1u < Meff && s != smax && s + 1u != smax) {
                    const uint32_t p = L.par[s];
                    if (p != RLC_NONE && p == L.par[s + 1u]) {
                        pair_ok = true;
                        pbits = __float_as_uint(L.Q[s] + L.Q[s + 1u]);
                    }
                }
                const uint32_t pmin = __reduce_min_sync(~0ull, pbits);
                const unsigned long long at_min = __ballot(pair_ok && pbits == pmin);
                if (smax != RLC_NONE && at_min) {
                    smin = (uint32_t)__ffsll((long long)at_min) - 1u;
                    qpmin = __uint_as_float(pmin);
                    changed = L.Q[smax] > ap.T * qpmin;
                }
            } else {
                // l_max: largest Q among splittable cut nodes, ties -> smallest slot
                unsigned long long best = 0ull;
#pragma unroll
                for (int j = 0; j < PER; ++j) {
                    uint32_t s = lane + kWave * j;
                    if (s < Meff) {
                        // a cluster of two or more lights is an internal node
                        if (L.end[s] - (s ? L.end[s - 1u] : 0u) > 1u) {
                            unsigned long long key = ((unsigned long long)__float_as_uint(L.Q[s]) << 32) |
                                                     (unsigned long long)(0xFFFFFFFFu - s);
                            best = key > best ? key : best;
                        }
                    }
                }
                best = wave_max_u64(best);
                if (best != 0ull) smax = 0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull);
                // p_min: sibling pairs (s, s+1) not holding l_max, smallest Q sum
                unsigned long long worst = ~0ull;
#pragma unroll
                for (int j = 0; j < PER; ++j) {
                    uint32_t s = lane + kWave * j;
                    if (s + 1u < Meff && s != smax && s + 1u != smax) {
                        // neighbouring cut nodes with one parent are its two children
                        const uint32_t p = L.par[s];
                        if (p != RLC_NONE && p == L.par[s + 1u]) {
                            float qp = L.Q[s] + L.Q[s + 1u];
                            unsigned long long key = ((unsigned long long)__float_as_uint(qp) << 32) | s;
                            worst = key < worst ? key : worst;
                        }
                    }
                }
                worst = wave_min_u64(worst);
                if (smax != RLC_NONE && worst != ~0ull) {
                    smin = (uint32_t)(worst & 0xFFFFFFFFull);
                    qpmin = __uint_as_float((uint32_t)(worst >> 32));
                    changed = L.Q[smax] > ap.T * qpmin;
                }
            }
            if (!changed) break;
            // new slot of old slot s: s + [s > smax] - [s > smin + 1]
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                uint32_t s = lane + kWave * j;
                if (s < Meff && s != smin + 1u) {
                    uint32_t nd = L.node[s];
                    float q = L.Q[s];
                    uint32_t dst = s + (s > smax ? 1u : 0u) - (s > smin + 1u ? 1u : 0u);
                    if (s == smin) {
                        // the parent covers both children: it ends where the right one does
                        L.nnode[dst] = L.par[s];
                        L.nend[dst] = L.end[s + 1u];
                        L.nQ[dst] = qpmin;
                        if (more) L.npar[dst] = ap.tree.parent[L.par[s]];
                    } else if (s == smax) {
                        // the first step splits a node of the loaded cut,
                        // whose children and split point came with it
                        float h = 0.5f * q;
                        const bool pre = step == 0u;
                        const uint32_t lc = pre ? pre_l[j] : ap.tree.left[nd];
                        L.nnode[dst] = lc;
                        L.nend[dst] = pre ? pre_sp[j] : ap.tree.last[lc] + 1u;
                        L.nQ[dst] = h;
                        L.nnode[dst + 1u] = pre ? pre_r[j] : ap.tree.right[nd];
                        L.nend[dst + 1u] = L.end[s];
                        L.nQ[dst + 1u] = h;
                        if (more) L.npar[dst] = L.npar[dst + 1u] = nd;
                    } else {
                        L.nnode[dst] = nd;
                        L.nend[dst] = L.end[s];
                        L.nQ[dst] = q;
                        if (more) L.npar[dst] = L.par[s];
                    }
                }
            }
            wave_sync();
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                uint32_t s = lane + kWave * j;
                if (s < Meff) {
                    L.node[s] = L.nnode[s];
                    L.end[s] = L.nend[s];
                    L.Q[s] = L.nQ[s];
                    if (more) L.par[s] = L.npar[s];
                }
            }
            wave_sync();
        }
    }
    wave_sync();
    return true;
}

// Q~ and Eq. 2 of one cell by the calling lane alone, from L.Q: sums taken
// left to right.
__device__ __forceinline__ void eq2_one_lane(const AdaptParams& ap, const AdaptLds& L, uint32_t Meff) {
    float S = 0.0f;
    for (uint32_t s = 0; s < Meff; ++s) S = S + L.Q[s];
    float acc = 0.0f;
    if (S == 0.0f) {
        for (uint32_t s = 0; s < Meff; ++s) {
            L.Qt[s] = 1.0f;
            acc = s ? acc + 1.0f : 1.0f;
            L.C[s] = acc;
        }
    } else {
        const float fl = eq2_floor(ap, S, Meff);
        for (uint32_t s = 0; s < Meff; ++s) {
            float qt = L.Q[s] + fl;
            L.Qt[s] = qt;
            acc = s ? acc + qt : qt;
            L.C[s] = acc;
        }
    }
}

// Q~ and Eq. 2 by lane 0 of the wave: sums taken left to right.
template <int PER>
__device__ __forceinline__ void adapt_eq2(const AdaptParams& ap, const AdaptLds& L) {
    const uint32_t lane = threadIdx.x & (kWave - 1u);
    const uint32_t Meff = ap.tmpl.Meff;
    float myq = 0.0f;
    if constexpr (PER == 1) myq = lane < Meff ? L.Q[lane] : 0.0f;
    if (lane == 0) {
        if constexpr (PER == 1) {
            // every slot's Q sits in its lane's register; lane 0 reads them in
            // slot order (a cross-lane register read, no LDS round trip)
            float S = 0.0f;
            for (uint32_t s = 0; s < Meff; ++s) S = S + lane_value(myq, s);
            float acc = 0.0f;
            if (S == 0.0f) {
                for (uint32_t s = 0; s < Meff; ++s) {
                    L.Qt[s] = 1.0f;
                    acc = s ? acc + 1.0f : 1.0f;
                    L.C[s] = acc;
                }
            } else {
                const float fl = eq2_floor(ap, S, Meff);
                for (uint32_t s = 0; s < Meff; ++s) {
                    const float qt = lane_value(myq, s) + fl;
                    L.Qt[s] = qt;
                    acc = s ? acc + qt : qt;
                    L.C[s] = acc;
                }
            }
        } else {
            eq2_one_lane(ap, L, Meff);
        }
    }
    wave_sync();
}

// The back: the cell's new tables from L to the cell table, statistics
// cleared, the cell marked ready.
template <int PER>
__device__ __forceinline__ void adapt_back(const AdaptParams& ap, uint32_t c, const AdaptLds& L) {
    const DevCells& cells = ap.cells;
    const uint32_t lane = threadIdx.x & (kWave - 1u);
    const uint32_t Meff = ap.tmpl.Meff;
    const size_t base = (size_t)c * cells.M;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        uint32_t s = lane + kWave * j;
        if (s < Meff) {
            cells.node[base + s] = L.node[s];
            cells.end[base + s] = L.end[s];
            cells.Q[base + s] = L.Q[s];
            cells.Qt[base + s] = L.Qt[s];
            cells.C[base + s] = L.C[s];
            cells.sum[base + s] = 0ull;
            cells.cnt[base + s] = 0u;
        }
    }
    if (lane == 0) cells.ready[c] = 1u;
    wave_sync();
}

// The rows in use: row k * stripes + s for k below stripe s's count.  They
// lie in rows 0 .. span - 1 (span: the largest count times the stripes),
// with a few unused rows where a stripe has fewer cells than the fullest.
// Built by one wave (lane s reads stripe s's counter, then a maximum across
// the lanes).
struct RowMap {
    uint32_t used[RLC_ROW_STRIPES_MAX];
    uint32_t span;
    uint32_t shift;  // log2(stripes)
};

__device__ __forceinline__ void row_map_build(const DevCells& c, RowMap& m) {
    const uint32_t lane = threadIdx.x & (kWave - 1u);
    uint32_t v = 0;
    if (lane < c.stripes) {
        const uint32_t n = c.n_live[lane * RLC_NLIVE_STRIDE];
        v = n < c.stripe_rows ? n : c.stripe_rows;
        m.used[lane] = v;
    }
    uint32_t mx = v;
#pragma unroll
    for (int off = 1; off < (int)kWave; off <<= 1) {
        const uint32_t t = (uint32_t)__shfl_xor((int)mx, off, kWave);
        mx = t > mx ? t : mx;
    }
    if (lane == 0) {
        m.span = mx * c.stripes;
        m.shift = (uint32_t)__builtin_ctz(c.stripes);
    }
}

__device__ __forceinline__ bool row_used(const DevCells& c, const RowMap& m, uint32_t r) {
    return r < m.span && (r >> m.shift) < m.used[r & (c.stripes - 1u)];
}

// The cells of rows li, li + grid, ...: each cell's loads are issued before
// the previous cell's work (with one slot per lane; four slots per lane
// would hold too many registers).
template <int PER>
__device__ __forceinline__ void adapt_cells(const AdaptParams& ap, const AdaptLds& L, RowMap& map) {
    row_map_build(ap.cells, map);
    wave_sync();
    const uint32_t span = map.span;
    // the rows this block visits (stride: the grid), unused ones skipped
    auto next_row = [&](uint32_t r) {
        while (r < span && !row_used(ap.cells, map, r)) r += gridDim.x;
        return r;
    };
    uint32_t li = next_row(blockIdx.x);
    if (li < span) {
        CellIn<PER> cur, nxt;
        load_cell<PER>(ap, li, cur);
        load_cell_nodes<PER>(ap, cur);
        while (li < span) {
            const uint32_t ln = next_row(li + gridDim.x);
            if (PER == 1 && ln < span) load_cell<PER>(ap, ln, nxt);
            const bool active = adapt_front<PER>(ap, cur, L);
            // the next cell's node records, once its row has arrived
            if (PER == 1 && ln < span) load_cell_nodes<PER>(ap, nxt);
            if (active) {
                adapt_eq2<PER>(ap, L);
                adapt_back<PER>(ap, cur.c, L);
            }
            if (ln < span) {
                if (PER == 1) {
                    cur = nxt;
                } else {
                    load_cell<PER>(ap, ln, cur);
                    load_cell_nodes<PER>(ap, cur);
                }
            }
            li = ln;
        }
    }
    wave_sync();  // the map is rebuilt by the next call (the batch's next scene)
}

// One block = one wavefront; it walks the list of created cells.  The LDS
// scratch is sized for the cut (8 arrays of 64 PER words).
template <int PER>
__global__ void __launch_bounds__(kWave, PER == 1 ? 8 : 4) k_adapt(AdaptParams /* read in place */) {
    const AdaptParams& ap = first_kernel_arg<AdaptParams>();
    extern __shared__ uint32_t lds[];
    __shared__ RowMap s_map;
    const AdaptLds L = lds_view(lds, kWave * PER);
    adapt_cells<PER>(ap, L, s_map);
}

// The same over every scene of a batch.
template <int PER>
__global__ void __launch_bounds__(kWave, PER == 1 ? 8 : 4) k_batch_adapt(const AdaptParams* __restrict__ aps, uint32_t n_scenes) {
    extern __shared__ uint32_t lds[];
    __shared__ RowMap s_map;
    const AdaptLds L = lds_view(lds, kWave * PER);
    typedef const __attribute__((address_space(4))) AdaptParams* ConstAdaptParams;
    for (uint32_t sc = 0; sc < n_scenes; ++sc) {
        const AdaptParams& ap = opaque_const((ConstAdaptParams)uniform_u64((uint64_t)&aps[sc]));
        adapt_cells<PER>(ap, L, s_map);
    }
}

// The fused kernel's blocks for the next pass, longest first: a counting
// sort of the n blocks' recorded durations into kOrderBuckets equal ranges
// between the shortest and the longest, by one workgroup of kOrderThreads
// threads (blocks in one range in no particular order).  Each wave counts
// into its own histogram, so the LDS atomics of a range queue only within a
// wave.  s: kOrderLds words of LDS.
constexpr uint32_t kOrderBuckets = 256;
constexpr uint32_t kOrderThreads = 1024;
constexpr uint32_t kOrderWaves = kOrderThreads / kWave;
constexpr uint32_t kOrderLds = (kOrderWaves + 1u) * kOrderBuckets + 2u;

// Range of duration c, counted from the longest (a float product: the same
// key wherever it is computed, which is all the sort needs).
__device__ __forceinline__ uint32_t order_key(uint32_t c, uint32_t lo, float scale) {
    const uint32_t k = (uint32_t)((float)(c - lo) * scale);
    return kOrderBuckets - 1u - (k < kOrderBuckets - 1u ? k : kOrderBuckets - 1u);
}

__device__ __forceinline__ void block_order(const uint32_t* __restrict__ cost, uint32_t* __restrict__ order,
                                            uint32_t n, uint32_t* s) {
    const uint32_t t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    uint32_t* hist = s;                                  // [wave][bucket]
    uint32_t* tot = s + kOrderWaves * kOrderBuckets;     // per bucket: count, then first position
    uint32_t* ext = tot + kOrderBuckets;                 // [0] shortest, [1] longest
    for (uint32_t j = t; j < kOrderWaves * kOrderBuckets; j += kOrderThreads) hist[j] = 0u;
    if (t == 0) {
        ext[0] = 0xFFFFFFFFu;
        ext[1] = 0u;
    }
    __syncthreads();
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (uint32_t i = t; i < n; i += kOrderThreads) {
        const uint32_t c = cost[i];
        lo = c < lo ? c : lo;
        hi = c > hi ? c : hi;
    }
#pragma unroll
    for (int off = 1; off < (int)kWave; off <<= 1) {
        const uint32_t a = (uint32_t)__shfl_xor((int)lo, off, kWave), b = (uint32_t)__shfl_xor((int)hi, off, kWave);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    if (lane == 0) {
        atomicMin(&ext[0], lo);
        atomicMax(&ext[1], hi);
    }
    __syncthreads();
    lo = ext[0];
    const float scale = (float)kOrderBuckets / ((float)(ext[1] - lo) + 1.0f);
    uint32_t* mine = hist + wave * kOrderBuckets;
    for (uint32_t i = t; i < n; i += kOrderThreads) atomicAdd(&mine[order_key(cost[i], lo, scale)], 1u);
    __syncthreads();
    // per bucket: each wave's count becomes the count of the waves before it
    if (t < kOrderBuckets) {
        uint32_t run = 0;
        for (uint32_t w = 0; w < kOrderWaves; ++w) {
            const uint32_t v = hist[w * kOrderBuckets + t];
            hist[w * kOrderBuckets + t] = run;
            run += v;
        }
        tot[t] = run;
    }
    __syncthreads();
    if (t < kWave) {
        // exclusive scan of the buckets' counts, four buckets per lane
        constexpr uint32_t kPer = kOrderBuckets / kWave;
        uint32_t v[kPer], sum = 0;
#pragma unroll
        for (uint32_t k = 0; k < kPer; ++k) {
            v[k] = tot[t * kPer + k];
            sum += v[k];
        }
        uint32_t incl = sum;
#pragma unroll
        for (int off = 1; off < (int)kWave; off <<= 1) {
            const uint32_t u = (uint32_t)__shfl_up((int)incl, off, kWave);
            if (t >= (uint32_t)off) incl += u;
        }
        uint32_t at = incl - sum;
#pragma unroll
        for (uint32_t k = 0; k < kPer; ++k) {
            tot[t * kPer + k] = at;
            at += v[k];
        }
    }
    __syncthreads();
    if (t < kOrderBuckets)
        for (uint32_t w = 0; w < kOrderWaves; ++w) hist[w * kOrderBuckets + t] += tot[t];
    __syncthreads();
    for (uint32_t i = t; i < n; i += kOrderThreads) order[atomicAdd(&mine[order_key(cost[i], lo, scale)], 1u)] = i;
}

__global__ void __launch_bounds__(kOrderThreads) k_block_order(const uint32_t* __restrict__ cost,
                                                               uint32_t* __restrict__ order, uint32_t n) {
    __shared__ uint32_t s[kOrderLds];
    block_order(cost, order, n, s);
}

// Cuts of up to 64 clusters, 16 cells per block: one wavefront per cell
// for Eq. 1, split-collapse and the write-back, and, between two block
// barriers, one lane per cell for the serial sums of Eq. 2, so those sums
// are issued once for the block's 16 cells.  Every wave runs the same
// number of rounds, so all of them reach both barriers of every round.
constexpr uint32_t kCellWaves = 16;
// words of one wave's scratch, padded by one so that the serial phase's 16
// lanes, each in its own cell's scratch, read different LDS banks
constexpr uint32_t kCellRegion = kLdsArrays * kWave + 1u;
// blocks of the 16-cell kernels (the chip holds them all at once: two per
// compute unit)
constexpr uint32_t kAdaptBlocks = 512;
static_assert(kCellWaves * kWave == kOrderThreads, "the ordering block is one of the 16-cell kernel's");
static_assert(kCellWaves * kCellRegion >= kOrderLds, "LDS for the ordering block");

// With ap.blk_n > 0 the first block orders the fused kernel's blocks for the
// next pass, beside the cells' work (it is dispatched first, and the launch
// fits the chip at once, so it does not wait for a free compute unit), and
// the others take the cells.
__global__ void __launch_bounds__(kCellWaves * kWave, 8) k_adapt16(AdaptParams /* read in place */) {
    const AdaptParams& ap = first_kernel_arg<AdaptParams>();
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t s_active[kCellWaves];
    __shared__ RowMap s_map;
    const uint32_t first = ap.blk_n > 0u && ap.blk_n <= RLC_ORDER_MAX_BLOCKS ? 1u : 0u;
    if (blockIdx.x < first) {
        block_order(ap.blk_cost, ap.blk_order, ap.blk_n, lds);
        return;
    }
    const uint32_t blk = blockIdx.x - first, n_blk = kAdaptBlocks - first;
    const uint32_t wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const AdaptLds L = lds_view(lds + wave * kCellRegion, kWave);
    // each round's cell is loaded during the round before (a launch
    // touches every cell once, so no round writes the next one's cell); the
    // first round's row before the row map says whether it is in use (every
    // row of the pool is allocated, and an unused row's data is not used)
    CellIn<1> nxt;
    const uint32_t li0 = blk * kCellWaves + wave;
    if (li0 < ap.cells.rows) load_cell<1>(ap, li0, nxt);
    if (wave == 0) row_map_build(ap.cells, s_map);
    __syncthreads();
    if (row_used(ap.cells, s_map, li0)) load_cell_nodes<1>(ap, nxt);
    const uint32_t n_live = s_map.span;
    const uint32_t per_round = n_blk * kCellWaves;
    const uint32_t rounds = (n_live + per_round - 1u) / per_round;
    for (uint32_t rd = 0; rd < rounds; ++rd) {
        const uint32_t li = rd * per_round + li0;
        bool active = false;
        uint32_t c = 0;
        const CellIn<1> in = nxt;
        if (row_used(ap.cells, s_map, li + per_round)) load_cell<1>(ap, li + per_round, nxt);
        if (row_used(ap.cells, s_map, li)) {
            c = in.c;
            active = adapt_front<1>(ap, in, L);
        }
        // the next round's node records, once its row has arrived
        if (row_used(ap.cells, s_map, li + per_round)) load_cell_nodes<1>(ap, nxt);
        if (lane == 0) s_active[wave] = active ? 1u : 0u;
        __syncthreads();
        if (wave == 0 && lane < kCellWaves && s_active[lane])
            eq2_one_lane(ap, lds_view(lds + lane * kCellRegion, kWave), ap.tmpl.Meff);
        __syncthreads();
        if (active) adapt_back<1>(ap, c, L);
    }
}

// The end of pass of a batch's cells (up to kBatchScenes16 scenes), 16 per
// block as in k_adapt16, over one index space of all scenes' rows in use:
// entry j is scene sc's entry j - off[sc], and a scene's entries run
// through its stripes in turn (stripe s's rows k * stripes + s, k below its
// count).  Every block stages the scenes' per-stripe prefix sums in LDS;
// each wave maps its next cell's entry during the current round.  A round's
// 16 cells may belong to different scenes, so each wave reads its own
// scene's parameters, and in the serial phase each lane its cell's scene's.
// The same arithmetic as k_adapt16, cell for cell.
constexpr uint32_t kBatchScenes16 = 16;

__global__ void __launch_bounds__(kCellWaves * kWave, 8) k_batch_adapt16(const AdaptParams* __restrict__ aps,
                                                                        uint32_t n_scenes) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t s_active[kCellWaves];
    __shared__ uint32_t s_scene[kCellWaves];
    // per scene: the rows in use before each stripe, and the total at [64]
    __shared__ uint32_t s_pref[kBatchScenes16][RLC_ROW_STRIPES_MAX + 1];
    __shared__ uint32_t s_off[kBatchScenes16 + 1];
    typedef const __attribute__((address_space(4))) AdaptParams* ConstAdaptParams;
    const uint32_t wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const AdaptLds L = lds_view(lds + wave * kCellRegion, kWave);
    auto params = [&](uint32_t sc) -> const AdaptParams& {
        return opaque_const((ConstAdaptParams)uniform_u64((uint64_t)&aps[sc]));
    };
    if (wave < n_scenes) {
        // wave w: scene w's counts, scanned across the lanes (lane = stripe)
        const DevCells& c = params(wave).cells;
        uint32_t v = 0;
        if (lane < c.stripes) {
            const uint32_t nl = c.n_live[lane * RLC_NLIVE_STRIDE];
            v = nl < c.stripe_rows ? nl : c.stripe_rows;
        }
#pragma unroll
        for (int off = 1; off < (int)kWave; off <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)v, off, kWave);
            if (lane >= (uint32_t)off) v += t;
        }
        s_pref[wave][lane + 1u] = v;
        if (lane == 0) s_pref[wave][0] = 0u;
    }
    __syncthreads();
    if (wave == 0) {
        uint32_t v = lane < n_scenes ? s_pref[lane][RLC_ROW_STRIPES_MAX] : 0u;
#pragma unroll
        for (int off = 1; off < (int)kBatchScenes16; off <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)v, off, kWave);
            if (lane >= (uint32_t)off) v += t;
        }
        if (lane < kBatchScenes16) s_off[lane + 1u] = v;
        if (lane == 0) s_off[0] = 0u;
    }
    __syncthreads();
    const uint32_t n = s_off[n_scenes];
    // entry j -> (scene, row) by two binary searches in LDS (the last scene,
    // then the last stripe, whose offset is at most j: empty ones are
    // passed over); j is the same for every lane of the wave
    auto locate = [&](uint32_t j, uint32_t& sc, uint32_t& row) {
        uint32_t lo = 0, hi = n_scenes - 1u;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1u) >> 1;
            if (s_off[mid] <= j)
                lo = mid;
            else
                hi = mid - 1u;
        }
        sc = lo;
        const uint32_t jj = j - s_off[sc];
        lo = 0;
        hi = RLC_ROW_STRIPES_MAX - 1u;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1u) >> 1;
            if (s_pref[sc][mid] <= jj)
                lo = mid;
            else
                hi = mid - 1u;
        }
        row = (jj - s_pref[sc][lo]) * params(sc).cells.stripes + lo;
    };
    const uint32_t per_round = gridDim.x * kCellWaves;
    const uint32_t rounds = (n + per_round - 1u) / per_round;
    const uint32_t li0 = blockIdx.x * kCellWaves + wave;
    // each round's cell is loaded during the round before, as in k_adapt16,
    // and the entry after it located in the round before that, while the
    // block waits for the serial sums
    CellIn<1> nxt;
    uint32_t sc_nxt = 0, sc_far = 0, row_far = 0;
    if (li0 < n) {
        uint32_t row;
        locate(li0, sc_nxt, row);
        load_cell<1>(params(sc_nxt), row, nxt);
        load_cell_nodes<1>(params(sc_nxt), nxt);
    }
    if (li0 + per_round < n) locate(li0 + per_round, sc_far, row_far);
    for (uint32_t rd = 0; rd < rounds; ++rd) {
        const uint32_t li = rd * per_round + li0;
        const uint32_t ln = li + per_round, lf = ln + per_round;
        bool active = false;
        uint32_t c = 0;
        const CellIn<1> in = nxt;
        const uint32_t sc = sc_nxt;
        if (ln < n) {
            sc_nxt = sc_far;
            load_cell<1>(params(sc_nxt), row_far, nxt);
        }
        if (li < n) {
            c = in.c;
            active = adapt_front<1>(params(sc), in, L);
        }
        // the next round's node records, once its row has arrived
        if (ln < n) load_cell_nodes<1>(params(sc_nxt), nxt);
        if (lane == 0) {
            s_active[wave] = active ? 1u : 0u;
            s_scene[wave] = sc;
        }
        __syncthreads();
        if (wave == 0) {
            if (lane < kCellWaves && s_active[lane]) {
                const AdaptParams& apl = aps[s_scene[lane]];
                eq2_one_lane(apl, lds_view(lds + lane * kCellRegion, kWave), apl.tmpl.Meff);
            }
        } else if (lf < n) {
            locate(lf, sc_far, row_far);
        }
        __syncthreads();
        if (wave == 0 && lf < n) locate(lf, sc_far, row_far);
        if (active) adapt_back<1>(params(sc), c, L);
    }
}

// Checkpoint load: one wavefront per cell.  The cell is found (or created)
// by its key, its cut and Q are taken as given, the ends follow from the
// tree, Q~ and C from Eq. 2 as at the end of a pass, and the write-back
// clears the statistics and marks the cell ready.  The host has checked
// that every cut is a partition of the lights.
template <int PER>
__global__ void __launch_bounds__(kWave) k_load_cells(AdaptParams /* read in place */,
                                                      const unsigned long long* __restrict__ keys,
                                                      const uint32_t* __restrict__ node, const float* __restrict__ Q,
                                                      uint32_t n, uint32_t* err) {
    const AdaptParams& ap = first_kernel_arg<AdaptParams>();
    extern __shared__ uint32_t lds[];
    const AdaptLds L = lds_view(lds, kWave * PER);
    const uint32_t lane = threadIdx.x & (kWave - 1u);
    const uint32_t Meff = ap.tmpl.Meff;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const unsigned long long key = keys[i];
        uint32_t row = RLC_NONE;
        if (lane == 0) row = find_or_create(ap.cells, key, (uint32_t)(key & 0xFFFFFFFFull), err);
        row = (uint32_t)__shfl((int)row, 0, kWave);
        if (row == RLC_NONE) continue;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t s = lane + kWave * j;
            if (s < Meff) {
                const uint32_t nd = node[(size_t)i * Meff + s];
                L.node[s] = nd;
                L.end[s] = ap.tree.last[nd] + 1u;
                L.Q[s] = Q[(size_t)i * Meff + s];
            }
        }
        wave_sync();
        if (lane == 0) eq2_one_lane(ap, L, Meff);
        wave_sync();
        adapt_back<PER>(ap, row, L);
    }
}

__global__ void k_gather_cells(DevCells c, uint32_t Meff, const uint32_t* __restrict__ rows, uint32_t n,
                               uint32_t* node, uint32_t* end, float* Q, float* Qt, float* C,
                               unsigned long long* sum, uint32_t* cnt) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)n * Meff) return;
    size_t row = i / Meff, s = i % Meff;
    size_t src = (size_t)rows[row] * c.M + s;
    if (node) node[i] = c.node[src];
    if (end) end[i] = c.end[src];
    if (Q) Q[i] = c.Q[src];
    if (Qt) Qt[i] = c.Qt[src];
    if (C) C[i] = c.C[src];
    if (sum) sum[i] = c.sum[src];
    if (cnt) cnt[i] = c.cnt[src];
}

}  // namespace

hipError_t launch_batch_adapt16(const AdaptParams* aps, uint32_t n_scenes, hipStream_t s) {
    if (n_scenes == 0 || n_scenes > kBatchScenes16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_adapt16, dim3(512), dim3(kCellWaves * kWave), kCellWaves * kCellRegion * 4, s, aps,
                       n_scenes);
    return hipGetLastError();
}

hipError_t launch_batch_adapt(const AdaptParams* aps, uint32_t n_scenes, uint32_t Meff, hipStream_t s) {
    if (Meff <= (uint32_t)kWave)
        hipLaunchKernelGGL(k_batch_adapt<1>, dim3(8192), dim3(kWave), kLdsArrays * kWave * 4, s, aps, n_scenes);
    else
        hipLaunchKernelGGL(k_batch_adapt<kMaxPerLane>, dim3(8192), dim3(kWave), kLdsArrays * RLC_MMAX * 4, s, aps,
                           n_scenes);
    return hipGetLastError();
}

hipError_t launch_adapt(const AdaptParams& ap, hipStream_t s) {
    // enough waves to fill the chip (8 per SIMD); each walks the list of
    // created cells with a stride of the grid size.  With repeated
    // split-collapse steps the cells of a 16-cell block take different
    // numbers of steps and the block waits for its slowest, so those passes
    // take the one-wave kernel.
    const bool order = ap.blk_n > 0u && ap.blk_n <= RLC_ORDER_MAX_BLOCKS;
    if (ap.tmpl.Meff <= (uint32_t)kWave && ap.split_steps <= 1u) {
        // the ordering block rides along with the cells' blocks
        hipLaunchKernelGGL(k_adapt16, dim3(kAdaptBlocks), dim3(kCellWaves * kWave), kCellWaves * kCellRegion * 4, s,
                           ap);
        return hipGetLastError();
    }
    if (order) hipLaunchKernelGGL(k_block_order, dim3(1), dim3(kOrderThreads), 0, s, ap.blk_cost, ap.blk_order, ap.blk_n);
    if (ap.tmpl.Meff <= (uint32_t)kWave)
        hipLaunchKernelGGL(k_adapt<1>, dim3(8192), dim3(kWave), kLdsArrays * kWave * 4, s, ap);
    else
        hipLaunchKernelGGL(k_adapt<kMaxPerLane>, dim3(8192), dim3(kWave), kLdsArrays * RLC_MMAX * 4, s, ap);
    return hipGetLastError();
}

hipError_t launch_load_cells(const AdaptParams& ap, const unsigned long long* keys, const uint32_t* node,
                             const float* Q, uint32_t n, uint32_t* err, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t grid = n < 4096u ? n : 4096u;
    if (ap.tmpl.Meff <= (uint32_t)kWave)
        hipLaunchKernelGGL(k_load_cells<1>, dim3(grid), dim3(kWave), kLdsArrays * kWave * 4, s, ap, keys, node, Q, n,
                           err);
    else
        hipLaunchKernelGGL(k_load_cells<kMaxPerLane>, dim3(grid), dim3(kWave), kLdsArrays * RLC_MMAX * 4, s, ap, keys,
                           node, Q, n, err);
    return hipGetLastError();
}

hipError_t launch_gather_cells(DevCells c, uint32_t Meff, const uint32_t* rows, uint32_t n, uint32_t* node,
                               uint32_t* end, float* Q, float* Qt, float* C, unsigned long long* sum,
                               uint32_t* cnt, hipStream_t s) {
    size_t total = (size_t)n * Meff;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_cells, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, s, c, Meff, rows, n,
                       node, end, Q, Qt, C, sum, cnt);
    return hipGetLastError();
}

}  // namespace rlc
