// C ABI of librlc (declared in include/rlc.h): argument checks, ownership of
// the library's device buffers, and the order of kernel launches for each
// call.  No exception leaves this file.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "mlp_internal.h"

using namespace rlc;

// Device memory of rlc_frame_sub_noalloc, for callers that cannot allocate:
// the radiance of one sub-frame pass, 3 floats per point.  Every GPU the
// library runs on holds its own copy until the process ends.  In host code
// this name is not a device address: the address comes from
// hipGetSymbolAddress with the device current (scratch_for_device).
static __device__ __align__(256) float scratch[3u * RLC_NOALLOC_MAX_POINTS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The address of the current device's scratch array (`dev` must be the
// current device), looked up once per device.
int scratch_for_device(int dev, float** out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return RLC_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return RLC_EHIP;
        }
        g_scratch_ptr[dev] = static_cast<float*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return RLC_OK;
}

}  // namespace

struct rlc_ctx {
    rlc_config cfg;
    hipStream_t stream = nullptr;
    char msg[512] = {0};

    // reference tree and initial cut
    bool tree_built = false;
    uint32_t N = 0, Meff = 0;
    float4* rec = nullptr;
    uint32_t* perm = nullptr;
    uint32_t* rank = nullptr;  // sorted position of each input light
    uint32_t* morton = nullptr;
    uint32_t* left = nullptr;
    uint32_t* right = nullptr;
    uint32_t* parent = nullptr;
    uint32_t* first = nullptr;
    uint32_t* last = nullptr;
    uint32_t* inode = nullptr;  // 4 words per internal node (left, right, split, parent)
    uint32_t* tmpl_node = nullptr;
    uint32_t* tmpl_end = nullptr;
    float* tmpl_Qt = nullptr;
    float* tmpl_C = nullptr;

    // occluders
    bool occ_set = false;
    uint32_t K = 0;
    float4* box = nullptr;
    uint32_t* occ_head = nullptr;
    uint32_t* occ_ref = nullptr;
    DevOcc occ{};

    // radiance of one sub-frame pass (rlc_frame_sub), P x 3 floats
    float* sub_buf = nullptr;
    size_t sub_cap = 0;
    // the same for rlc_frame_sub_noalloc: this device's scratch array
    float* noalloc_scratch = nullptr;

    // fused-kernel block scheduling: each block's duration in the last pass,
    // the longest-first order built from it, and the block count that order
    // is for (0: none yet)
    uint32_t* blk_cost = nullptr;
    uint32_t* blk_order = nullptr;
    uint32_t blk_ordered = 0;

    // cells
    DevCells cells{};
    uint32_t* d_err = nullptr;
    double* d_partial = nullptr;

    // derived constants
    uint64_t cell_index_limit = 0;   // linear cell indices are below this
    float inv_cell[3] = {0, 0, 0};
    float jit_reach[3] = {0, 0, 0};
    float f_r = 0.0f;
    float fx_scale = 1.0f, fx_inv = 1.0f;

    // learned proposal: fixed breadth-first cut of up to 64 nodes, FP32
    // master weights with Adam moments, BF16 operand fragments, scratch
    uint32_t fix_M = 0;
    uint32_t* fix_node = nullptr;
    uint32_t* fix_end = nullptr;
    float* fix_Qt = nullptr;
    float* fix_C = nullptr;
    bool mlp_ready = false;
    float* mlp_master = nullptr;
    float* mlp_m = nullptr;
    float* mlp_v = nullptr;
    uint16_t* mlp_frag = nullptr;
    uint32_t mlp_step = 0;
    double mlp_b1t = 1.0, mlp_b2t = 1.0;  // beta1^t, beta2^t after mlp_step steps
    float* mlp_partial = nullptr;
    uint32_t mlp_partial_blocks = 0;
    float* mlp_part_w = nullptr;
    float* mlp_part_loss = nullptr;
    float* mlp_loss = nullptr;
    uint16_t* mlp_xenc = nullptr;      // encoded inputs of the training call's points
    uint32_t mlp_xenc_cap = 0;
    // mixture with the learned proposal, and per-sample training records
    const float* mix_cdf = nullptr;
    uint32_t mix_rows = 0;
    // footprint-sized cells: per-point footprints (caller memory), the
    // finest cell edge and the first linear index of every level
    const float* fp_arr = nullptr;
    uint32_t fp_rows = 0;
    float fp_base = 0.0f;
    uint32_t lvl_first[RLC_MAX_LEVELS + 1] = {0};
    float mix_w = 0.5f;
    uint32_t* log_pid = nullptr;
    uint32_t* log_node = nullptr;
    float* log_w = nullptr;
    uint64_t log_cap = 0;

    // batches built over this context: their captured graphs hold the
    // context's buffer addresses, so rebuilding the tree or the occluders
    // bumps the generation (the batch recaptures), and the context cannot be
    // destroyed while a batch refers to it
    uint32_t generation = 0;
    uint32_t batch_refs = 0;

    // per-kernel timing
    bool timing = false;
    std::vector<hipEvent_t> pending;   // 3 per timed frame
    std::vector<hipEvent_t> mlp_pending;  // 3 per timed training step
    std::vector<hipEvent_t> spare;
    hipEvent_t join = nullptr;  // marks this stream's work for another context's stream to wait on
};

namespace {

int fail(rlc_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->msg, sizeof(c->msg), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define RLC_HIP(ctx, call)                                                                         \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return fail((ctx), RLC_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <class T>
int dalloc(rlc_ctx* c, T** p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * n);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(c, RLC_ENOMEM, "hipMalloc of %zu bytes failed: %s", sizeof(T) * n, hipGetErrorString(e));
    }
    return RLC_OK;
}

template <class T>
void dfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

#define RLC_TRY(expr)            \
    do {                         \
        int r_ = (expr);         \
        if (r_ != RLC_OK) return r_; \
    } while (0)

bool finite_f(float v) { return std::isfinite(v); }

uint32_t blocks_for(size_t n, uint32_t b = 256) { return (uint32_t)((n + b - 1) / b); }

int reset_cells(rlc_ctx* c) {
    DevCells& d = c->cells;
    size_t bins = (size_t)d.rows * d.M;
    RLC_HIP(c, launch_fill_u64(d.keys, RLC_EMPTY_KEY, d.capacity, c->stream));
    RLC_HIP(c, launch_fill_u32(d.ready, 0u, d.rows, c->stream));
    RLC_HIP(c, launch_fill_u64(d.sum, 0ull, bins, c->stream));
    RLC_HIP(c, launch_fill_u32(d.cnt, 0u, bins, c->stream));
    RLC_HIP(c, launch_fill_u32(d.n_live, 0u, d.stripes * RLC_NLIVE_STRIDE, c->stream));
    return RLC_OK;
}

void free_tree(rlc_ctx* c) {
    dfree(c->rec);
    dfree(c->perm);
    dfree(c->rank);
    dfree(c->morton);
    dfree(c->left);
    dfree(c->right);
    dfree(c->parent);
    dfree(c->first);
    dfree(c->last);
    dfree(c->inode);
    dfree(c->tmpl_node);
    dfree(c->tmpl_end);
    dfree(c->tmpl_Qt);
    dfree(c->tmpl_C);
    dfree(c->fix_node);
    dfree(c->fix_end);
    dfree(c->fix_Qt);
    dfree(c->fix_C);
    c->fix_M = 0;
    c->mix_cdf = nullptr;
    c->mix_rows = 0;
    c->tree_built = false;
    c->generation += 1u;
}

void free_mlp(rlc_ctx* c) {
    dfree(c->mlp_master);
    dfree(c->mlp_m);
    dfree(c->mlp_v);
    dfree(c->mlp_frag);
    dfree(c->mlp_partial);
    dfree(c->mlp_part_w);
    dfree(c->mlp_part_loss);
    dfree(c->mlp_loss);
    dfree(c->mlp_xenc);
    c->mlp_xenc_cap = 0;
    c->mlp_partial_blocks = 0;
    c->mlp_ready = false;
}

void free_occ(rlc_ctx* c) {
    dfree(c->box);
    dfree(c->occ_head);
    dfree(c->occ_ref);
    c->occ = DevOcc{};
    c->occ_set = false;
    c->K = 0;
    c->generation += 1u;
}

DevTree dev_tree(const rlc_ctx* c) {
    DevTree t;
    t.rec = c->rec;
    t.left = c->left;
    t.right = c->right;
    t.parent = c->parent;
    t.first = c->first;
    t.last = c->last;
    t.inode = reinterpret_cast<const uint4*>(c->inode);
    t.N = c->N;
    return t;
}

DevCut dev_tmpl(const rlc_ctx* c) {
    DevCut t;
    t.node = c->tmpl_node;
    t.end = c->tmpl_end;
    t.Qt = c->tmpl_Qt;
    t.C = c->tmpl_C;
    t.Meff = c->Meff;
    return t;
}

FrameParams frame_params(const rlc_ctx* c) {
    FrameParams fp;
    fp.blk_order = nullptr;
    fp.blk_cost = nullptr;
    fp.tree = dev_tree(c);
    fp.tmpl = dev_tmpl(c);
    fp.cells = c->cells;
    fp.occ = c->occ;
    fp.occ.K = c->occ_set ? c->K : 0u;
    for (int a = 0; a < 3; ++a) {
        fp.grid_lo[a] = c->cfg.grid_lo[a];
        fp.inv_cell[a] = c->inv_cell[a];
        fp.dims[a] = c->cfg.grid_dims[a];
        fp.jit_reach[a] = c->jit_reach[a];
    }
    fp.normal_bits = c->cfg.normal_bits;
    fp.jitter = c->cfg.jitter;
    fp.scene_id = c->cfg.scene_id;
    fp.footprint = c->fp_arr;
    fp.fp_levels = c->cfg.footprint_levels > 1u ? c->cfg.footprint_levels : 1u;
    fp.fp_tile = c->cfg.footprint_tile;
    fp.fp_base = c->fp_base;
    for (uint32_t L = 0; L <= RLC_MAX_LEVELS; ++L) fp.lvl_first[L] = c->lvl_first[L];
    fp.seed_lo = (uint32_t)(c->cfg.seed & 0xFFFFFFFFull);
    fp.seed_hi = (uint32_t)(c->cfg.seed >> 32);
    fp.f_r = c->f_r;
    fp.t_lo = c->cfg.t_lo;
    fp.reward_max = c->cfg.reward_max;
    fp.fx_scale = c->fx_scale;
    fp.reward_mode = c->cfg.reward_mode;
    fp.two_sided = c->cfg.two_sided;
    fp.err = c->d_err;
    fp.mix_cdf = c->mix_cdf;
    fp.fix_end = c->fix_end;
    fp.fix_M = c->fix_M;
    fp.mix_w = c->mix_w;
    fp.log_pid = c->log_pid;
    fp.log_node = c->log_node;
    fp.log_w = c->log_w;
    return fp;
}

AdaptParams adapt_params(const rlc_ctx* c) {
    AdaptParams ap;
    ap.tree = dev_tree(c);
    ap.tmpl = dev_tmpl(c);
    ap.cells = c->cells;
    ap.alpha = c->cfg.alpha;
    ap.T = c->cfg.T;
    ap.eps = c->cfg.eps;
    ap.fx_inv = c->fx_inv;
    ap.adapt = c->cfg.adapt;
    ap.temporal = c->cfg.temporal;
    ap.split_steps = c->cfg.split_steps;
    ap.blk_cost = nullptr;
    ap.blk_order = nullptr;
    ap.blk_n = 0;
    return ap;
}

int need_tree(rlc_ctx* c) {
    if (!c) return RLC_EINVAL;
    if (!c->tree_built) return fail(c, RLC_ESTATE, "the light tree has not been built");
    return RLC_OK;
}

int check_frame_args(rlc_ctx* c, const void* pos, uint32_t P, uint32_t spp) {
    RLC_TRY(need_tree(c));
    if (P == 0) return RLC_OK;
    if (!pos) return fail(c, RLC_EINVAL, "null point array");
    if (spp == 0) return fail(c, RLC_EINVAL, "spp must be >= 1");
    if ((uint64_t)P * spp > 0xFFFFFFFFull) return fail(c, RLC_EINVAL, "P * spp exceeds 2^32 - 1");
    if (c->mix_cdf && P > c->mix_rows)
        return fail(c, RLC_EINVAL, "the mixture cdf has %u rows, the pass has %u points", c->mix_rows, P);
    if (c->fp_arr && P > c->fp_rows)
        return fail(c, RLC_EINVAL, "%u footprints are set, the pass has %u points", c->fp_rows, P);
    if (c->log_node && (uint64_t)P * spp > c->log_cap)
        return fail(c, RLC_EINVAL, "sample log holds %llu records, the pass has %llu",
                    (unsigned long long)c->log_cap, (unsigned long long)P * spp);
    return RLC_OK;
}

hipEvent_t take_event(rlc_ctx* c) {
    if (!c->spare.empty()) {
        hipEvent_t e = c->spare.back();
        c->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int read_device_errors(rlc_ctx* c) {
    uint32_t err = 0;
    RLC_HIP(c, hipMemcpyAsync(&err, c->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    RLC_HIP(c, hipStreamSynchronize(c->stream));
    if (err) {
        RLC_HIP(c, launch_fill_u32(c->d_err, 0u, 1, c->stream));
        RLC_HIP(c, hipStreamSynchronize(c->stream));
        if (err & RLC_DERR_CAPACITY)
            return fail(c, RLC_ECAPACITY,
                        "cell table full (rows for %u cells in %u stripes, %u lookup slots, or %u slots in a "
                        "row taken); some samples were not learned from",
                        c->cells.stripes * c->cells.stripe_rows, c->cells.stripes, c->cells.capacity,
                        RLC_HASH_MAX_PROBES);
        if (err & RLC_DERR_WAIT)
            return fail(c, RLC_EHIP, "a cell lookup gave up waiting for the cell's row to be published");
        if (err & RLC_DERR_FX_OVERFLOW)
            return fail(c, RLC_ECAPACITY,
                        "a fixed-point reward sum of one (cell, cluster) exceeded 64 bits in one pass: "
                        "lower fx_shift or reward_max; that pass's statistics are not valid");
        if (err & RLC_DERR_INPUT) return fail(c, RLC_EINVAL, "non-finite or inverted input");
        if (err & RLC_DERR_NONFINITE) return fail(c, RLC_EINVAL, "non-finite contribution");
    }
    return RLC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Learned proposal
// ---------------------------------------------------------------------------
namespace {

constexpr float kAdamBeta1 = 0.9f, kAdamBeta2 = 0.999f, kAdamEps = 1e-8f;

MlpEncode mlp_encode_params(const rlc_ctx* c) {
    MlpEncode e;
    for (int a = 0; a < 3; ++a) {
        e.lo[a] = c->cfg.grid_lo[a];
        e.ext[a] = c->cfg.grid_hi[a] - c->cfg.grid_lo[a];
    }
    return e;
}

int mlp_alloc(rlc_ctx* c) {
    if (c->mlp_master) return RLC_OK;
    RLC_TRY(dalloc(c, &c->mlp_master, kMlpParams));
    RLC_TRY(dalloc(c, &c->mlp_m, kMlpParams));
    RLC_TRY(dalloc(c, &c->mlp_v, kMlpParams));
    RLC_TRY(dalloc(c, &c->mlp_frag, 8 * (size_t)kMlpFragVecs));
    RLC_TRY(dalloc(c, &c->mlp_loss, 1));
    // the padding of the first layer's operands (inputs 144..159) stays zero
    RLC_HIP(c, hipMemsetAsync(c->mlp_frag, 0, sizeof(uint16_t) * 8 * (size_t)kMlpFragVecs, c->stream));
    return RLC_OK;
}

// New weights in master: zero Adam's state, refresh the BF16 operands.
int mlp_reset_optimizer(rlc_ctx* c) {
    RLC_HIP(c, hipMemsetAsync(c->mlp_m, 0, sizeof(float) * kMlpParams, c->stream));
    RLC_HIP(c, hipMemsetAsync(c->mlp_v, 0, sizeof(float) * kMlpParams, c->stream));
    RLC_HIP(c, launch_mlp_refresh(c->mlp_master, c->mlp_frag, c->stream));
    c->mlp_step = 0;
    c->mlp_b1t = 1.0;
    c->mlp_b2t = 1.0;
    c->mlp_ready = true;
    return RLC_OK;
}

int mlp_partials(rlc_ctx* c, uint32_t nblocks) {
    if (nblocks <= c->mlp_partial_blocks) return RLC_OK;
    dfree(c->mlp_partial);
    dfree(c->mlp_part_w);
    dfree(c->mlp_part_loss);
    c->mlp_partial_blocks = 0;
    RLC_TRY(dalloc(c, &c->mlp_partial, (size_t)nblocks * kMlpParams));
    RLC_TRY(dalloc(c, &c->mlp_part_w, nblocks));
    RLC_TRY(dalloc(c, &c->mlp_part_loss, nblocks));
    c->mlp_partial_blocks = nblocks;
    return RLC_OK;
}

// The training kernels read each point's encoded inputs from a buffer
// filled once per call (the points are shared by many tuples), for up to
// kMlpEncodeMaxPoints points (320 bytes each); beyond, the kernels encode.
constexpr uint32_t kMlpEncodeMaxPoints = 1u << 18;

int mlp_encoded_inputs(rlc_ctx* c, const float* pos, const float* nrm, uint32_t P, const uint16_t** out) {
    *out = nullptr;
    if (P > kMlpEncodeMaxPoints) return RLC_OK;
    if (P > c->mlp_xenc_cap) {
        RLC_HIP(c, hipStreamSynchronize(c->stream));
        dfree(c->mlp_xenc);
        c->mlp_xenc_cap = 0;
        RLC_TRY(dalloc(c, &c->mlp_xenc, (size_t)P * kMlpEncodeHalves));
        c->mlp_xenc_cap = P;
    }
    RLC_HIP(c, launch_mlp_encode(mlp_encode_params(c), pos, nrm, P, c->mlp_xenc, c->stream));
    *out = c->mlp_xenc;
    return RLC_OK;
}

int check_tuples(rlc_ctx* c, const float* pos, const float* nrm, uint32_t P, const uint32_t* pid,
                 const uint32_t* node, const float* w, uint32_t n) {
    RLC_TRY(need_tree(c));
    if (!c->mlp_ready) return fail(c, RLC_ESTATE, "the network has no weights (rlc_mlp_init / set_params)");
    if (n == 0) return RLC_OK;
    if (P == 0 || !pos || !nrm) return fail(c, RLC_EINVAL, "tuples need the points they refer to");
    if (!pid || !node || !w) return fail(c, RLC_EINVAL, "null tuple array");
    return RLC_OK;
}

}  // namespace

extern "C" {

const char* rlc_last_error(const rlc_ctx* ctx) { return ctx ? ctx->msg : "null context"; }

int rlc_create(const rlc_config* cfg, void* stream, rlc_ctx** out) {
    if (!out) return RLC_EINVAL;
    *out = nullptr;
    if (!cfg) return RLC_EINVAL;
    const rlc_config& k = *cfg;
    bool ok = k.M >= 1 && k.M <= RLC_MMAX && finite_f(k.alpha) && k.alpha >= 0.0f && k.alpha <= 1.0f &&
              finite_f(k.T) && k.T >= 0.0f && finite_f(k.eps) && k.eps >= 0.0f && k.fx_shift <= 40 &&
              finite_f(k.reward_max) && k.reward_max > 0.0f && finite_f(k.t_lo) && k.t_lo >= 0.0f &&
              k.t_lo < 0.5f && k.reward_mode <= 1 && finite_f(k.albedo) && k.albedo >= 0.0f &&
              k.occ_grid_res <= RLC_OCC_RES_MAX && k.split_steps <= RLC_SPLIT_STEPS_MAX && k.normal_bits <= 8 &&
              finite_f(k.jitter) && k.jitter >= 0.0f && k.jitter <= 1.0f && k.footprint_levels <= RLC_MAX_LEVELS &&
              (k.footprint_levels <= 1u || (finite_f(k.footprint_tile) && k.footprint_tile > 0.0f));
    for (int a = 0; a < 3; ++a)
        ok = ok && finite_f(k.grid_lo[a]) && finite_f(k.grid_hi[a]) && k.grid_hi[a] > k.grid_lo[a] &&
             k.grid_dims[a] >= 1 && k.grid_dims[a] <= (1u << 20);
    if (!ok) return RLC_EINVAL;
    // one clamped reward in fixed point must fit 63 bits (two of them may
    // wrap a sum: that is detected on the device and reported)
    if (std::ldexp((double)k.reward_max, (int)k.fx_shift) > 9223372036854775808.0) return RLC_EINVAL;
    // cells of the 5-D grid, positions times normal bins, over every level
    // of footprint-sized cells (level-major linear index: 32 bits)
    uint64_t lvl_first[RLC_MAX_LEVELS + 1] = {0};
    const uint32_t nlev = k.footprint_levels > 1u ? k.footprint_levels : 1u;
    for (uint32_t L = 0; L < nlev; ++L) {
        uint64_t cells = 1;
        for (int a = 0; a < 3; ++a) cells *= (uint64_t)(((k.grid_dims[a] - 1u) >> L) + 1u);
        lvl_first[L + 1] = lvl_first[L] + (cells << (2u * k.normal_bits));
    }
    for (uint32_t L = nlev + 1; L <= RLC_MAX_LEVELS; ++L) lvl_first[L] = lvl_first[nlev];
    const uint64_t dense = lvl_first[nlev];
    if (dense > 0xFFFFFFFFull) return RLC_EINVAL;
    uint64_t capacity;
    if (k.hashed) {
        if (k.capacity == 0 || k.capacity > (1u << 30)) return RLC_EINVAL;
        capacity = 64;
        while (capacity < k.capacity) capacity <<= 1;
    } else {
        if (dense > (1u << 28)) return RLC_EINVAL;
        capacity = dense;
    }
    if (k.max_cells > capacity) return RLC_EINVAL;
    const uint64_t pool = k.max_cells ? k.max_cells : capacity;
    if (pool * (uint64_t)k.M >= 0xFFFFFFFFull) return RLC_EINVAL;  // (cell, cluster) bins index with 32 bits
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RLC_EHIP;
    float* noalloc = nullptr;
    const int rs = scratch_for_device(dev, &noalloc);
    if (rs != RLC_OK) return rs;
    rlc_ctx* c = new (std::nothrow) rlc_ctx();
    if (!c) return RLC_ENOMEM;
    c->noalloc_scratch = noalloc;
    c->cfg = k;
    c->stream = (hipStream_t)stream;
    c->cell_index_limit = dense;
    for (uint32_t L = 0; L <= RLC_MAX_LEVELS; ++L) c->lvl_first[L] = (uint32_t)lvl_first[L];
    for (int a = 0; a < 3; ++a) {
        const float e = (k.grid_hi[a] - k.grid_lo[a]) / (float)k.grid_dims[a];
        if (a == 0 || e < c->fp_base) c->fp_base = e;
    }
    for (int a = 0; a < 3; ++a) {
        c->inv_cell[a] = (float)k.grid_dims[a] / (k.grid_hi[a] - k.grid_lo[a]);
        c->jit_reach[a] = k.jitter * ((k.grid_hi[a] - k.grid_lo[a]) / (float)k.grid_dims[a]);
    }
    c->f_r = (float)((double)k.albedo / 3.14159265358979323846);
    c->fx_scale = ldexpf(1.0f, (int)k.fx_shift);
    c->fx_inv = ldexpf(1.0f, -(int)k.fx_shift);
    DevCells& d = c->cells;
    d.capacity = (uint32_t)capacity;
    d.rows = (uint32_t)pool;
    // a pool of 4,096 rows or more is cut into stripes of about 1,024 rows
    // (a power of two of them, at most RLC_ROW_STRIPES_MAX), each with its
    // own row counter
    d.stripes = 1;
    while (d.stripes < RLC_ROW_STRIPES_MAX && pool >= 4096 && pool / (2u * d.stripes) >= 1024) d.stripes *= 2u;
    d.stripe_rows = (uint32_t)(pool / d.stripes);
    d.hashed = k.hashed ? 1u : 0u;
    d.M = k.M;
    size_t bins = (size_t)pool * k.M;
    int r = RLC_OK;
    if (r == RLC_OK) r = dalloc(c, &d.keys, capacity);
    if (r == RLC_OK) r = dalloc(c, &d.ready, pool);
    if (r == RLC_OK) r = dalloc(c, &d.node, bins);
    if (r == RLC_OK) r = dalloc(c, &d.end, bins);
    if (r == RLC_OK) r = dalloc(c, &d.Q, bins);
    if (r == RLC_OK) r = dalloc(c, &d.Qt, bins);
    if (r == RLC_OK) r = dalloc(c, &d.C, bins);
    if (r == RLC_OK) r = dalloc(c, &d.sum, bins);
    if (r == RLC_OK) r = dalloc(c, &d.cnt, bins);
    if (r == RLC_OK) r = dalloc(c, &d.live, pool);
    if (r == RLC_OK) r = dalloc(c, &d.n_live, RLC_ROW_STRIPES_MAX * RLC_NLIVE_STRIDE);
    if (r == RLC_OK) r = dalloc(c, &c->d_err, 1);
    if (r == RLC_OK) r = dalloc(c, &c->d_partial, 6 * 1024);
    if (r == RLC_OK) r = dalloc(c, &c->blk_cost, RLC_ORDER_MAX_BLOCKS);
    if (r == RLC_OK) r = dalloc(c, &c->blk_order, RLC_ORDER_MAX_BLOCKS);
    if (r == RLC_OK) r = reset_cells(c);
    if (r == RLC_OK) {
        hipError_t e = launch_fill_u32(c->d_err, 0u, 1, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) r = RLC_EHIP;
    }
    if (r != RLC_OK) {
        rlc_destroy(c);
        return r;
    }
    *out = c;
    return RLC_OK;
}

int rlc_destroy(rlc_ctx* c) {
    if (!c) return RLC_OK;
    if (c->batch_refs)
        return fail(c, RLC_ESTATE, "the context belongs to %u batch(es): destroy them first", c->batch_refs);
    (void)hipStreamSynchronize(c->stream);
    free_tree(c);
    free_occ(c);
    free_mlp(c);
    DevCells& d = c->cells;
    dfree(d.keys);
    dfree(d.ready);
    dfree(d.node);
    dfree(d.end);
    dfree(d.Q);
    dfree(d.Qt);
    dfree(d.C);
    dfree(d.sum);
    dfree(d.cnt);
    dfree(d.live);
    dfree(d.n_live);
    dfree(c->d_err);
    dfree(c->d_partial);
    dfree(c->blk_cost);
    dfree(c->blk_order);
    dfree(c->sub_buf);
    for (hipEvent_t e : c->pending) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->mlp_pending) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->spare) (void)hipEventDestroy(e);
    if (c->join) (void)hipEventDestroy(c->join);
    delete c;
    return RLC_OK;
}

int rlc_build_light_tree(rlc_ctx* c, const float* d_tri, const float* d_emit, uint32_t N) {
    if (!c) return RLC_EINVAL;
    if (!d_tri || !d_emit) return fail(c, RLC_EINVAL, "null triangle or emission array");
    if (N == 0) return fail(c, RLC_EINVAL, "N must be >= 1");
    if (N > (1u << 30)) return fail(c, RLC_EINVAL, "too many lights");
    RLC_HIP(c, hipStreamSynchronize(c->stream));
    free_tree(c);
    const uint32_t nn = 2u * N - 1u;
    const uint32_t M = c->cfg.M;
    RLC_TRY(dalloc(c, &c->rec, 4 * (size_t)N));
    RLC_TRY(dalloc(c, &c->perm, N));
    RLC_TRY(dalloc(c, &c->rank, N));
    RLC_TRY(dalloc(c, &c->morton, N));
    RLC_TRY(dalloc(c, &c->left, N > 1 ? N - 1 : 1));
    RLC_TRY(dalloc(c, &c->right, N > 1 ? N - 1 : 1));
    RLC_TRY(dalloc(c, &c->parent, nn));
    RLC_TRY(dalloc(c, &c->first, nn));
    RLC_TRY(dalloc(c, &c->last, nn));
    RLC_TRY(dalloc(c, &c->inode, 4 * (size_t)(N > 1 ? N - 1 : 1)));
    RLC_TRY(dalloc(c, &c->tmpl_node, M));
    RLC_TRY(dalloc(c, &c->tmpl_end, M));
    RLC_TRY(dalloc(c, &c->tmpl_Qt, M));
    RLC_TRY(dalloc(c, &c->tmpl_C, M));
    RLC_TRY(dalloc(c, &c->fix_node, RLC_MIX_M));
    RLC_TRY(dalloc(c, &c->fix_end, RLC_MIX_M));
    RLC_TRY(dalloc(c, &c->fix_Qt, RLC_MIX_M));
    RLC_TRY(dalloc(c, &c->fix_C, RLC_MIX_M));
    // temporaries
    float* sums = nullptr;
    float* part = nullptr;
    float* bbox = nullptr;
    uint32_t* ktmp = nullptr;
    uint32_t* vtmp = nullptr;
    uint32_t* hist = nullptr;
    uint32_t nb = std::min<uint32_t>(1024u, blocks_for(N));
    int r = RLC_OK;
    if (r == RLC_OK) r = dalloc(c, &sums, 3 * (size_t)N);
    if (r == RLC_OK) r = dalloc(c, &part, 6 * (size_t)nb);
    if (r == RLC_OK) r = dalloc(c, &bbox, 9);
    if (r == RLC_OK) r = dalloc(c, &ktmp, N);
    if (r == RLC_OK) r = dalloc(c, &vtmp, N);
    if (r == RLC_OK) r = dalloc(c, &hist, radix_sort_hist_entries(N));
    hipError_t e = hipSuccess;
    auto step = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    if (r == RLC_OK) {
        step(launch_fill_u32(c->d_err, 0u, 1, c->stream));
        step(launch_tri_prep(d_tri, N, sums, part, part + 3 * nb, nb, c->d_err, c->stream));
        step(launch_check_finite(d_emit, 3 * N, c->d_err, c->stream));
        step(launch_bbox_final(part, part + 3 * nb, nb, bbox, c->stream));
        step(launch_morton(sums, bbox, N, c->morton, c->perm, c->stream));
        step(radix_sort_pairs(c->morton, c->perm, ktmp, vtmp, hist, N, 30, c->stream));
        step(launch_gather_records(d_tri, d_emit, c->perm, N, c->rec, c->stream));
        step(launch_invert_perm(c->perm, N, c->rank, c->stream));
        step(launch_radix_tree(c->morton, c->perm, N, c->left, c->right, c->parent, c->first, c->last, c->inode,
                               c->stream));
        c->N = N;
        c->Meff = std::min(M, N);
        step(launch_initial_cut(dev_tree(c), M, c->tmpl_node, c->tmpl_end, c->tmpl_Qt, c->tmpl_C, c->stream));
        c->fix_M = std::min(RLC_MIX_M, N);
        step(launch_initial_cut(dev_tree(c), RLC_MIX_M, c->fix_node, c->fix_end, c->fix_Qt, c->fix_C, c->stream));
        step(hipStreamSynchronize(c->stream));
    }
    dfree(sums);
    dfree(part);
    dfree(bbox);
    dfree(ktmp);
    dfree(vtmp);
    dfree(hist);
    if (r != RLC_OK) return r;
    if (e != hipSuccess) return fail(c, RLC_EHIP, "light tree build: %s", hipGetErrorString(e));
    RLC_TRY(read_device_errors(c));
    c->tree_built = true;
    RLC_TRY(reset_cells(c));
    RLC_HIP(c, hipStreamSynchronize(c->stream));
    return RLC_OK;
}

int rlc_reset_cells(rlc_ctx* c) {
    if (!c) return RLC_EINVAL;
    return reset_cells(c);
}

int rlc_set_emission(rlc_ctx* c, const float* d_emit, uint32_t N) {
    RLC_TRY(need_tree(c));
    if (!d_emit) return fail(c, RLC_EINVAL, "null emission array");
    if (N != c->N) return fail(c, RLC_EINVAL, "emission for %u lights, tree has %u", N, c->N);
    RLC_HIP(c, launch_scatter_emission(d_emit, c->rank, N, c->rec, c->stream));
    return RLC_OK;
}

int rlc_set_occluders(rlc_ctx* c, const float* d_aabb, uint32_t K) {
    if (!c) return RLC_EINVAL;
    if (K && !d_aabb) return fail(c, RLC_EINVAL, "null box array");
    RLC_HIP(c, hipStreamSynchronize(c->stream));
    free_occ(c);
    if (K == 0) {
        c->occ_set = true;
        return RLC_OK;
    }
    uint32_t nb = std::min<uint32_t>(1024u, blocks_for(K));
    float* part = nullptr;
    RLC_TRY(dalloc(c, &c->box, 2 * (size_t)K));
    RLC_TRY(dalloc(c, &part, 6 * (size_t)nb));
    RLC_HIP(c, launch_fill_u32(c->d_err, 0u, 1, c->stream));
    RLC_HIP(c, launch_pack_boxes(d_aabb, K, c->box, part, part + 3 * nb, nb, c->d_err, c->stream));
    std::vector<float> hpart(6 * (size_t)nb);
    RLC_HIP(c, hipMemcpyAsync(hpart.data(), part, sizeof(float) * hpart.size(), hipMemcpyDeviceToHost, c->stream));
    RLC_HIP(c, hipStreamSynchronize(c->stream));
    dfree(part);
    int r = read_device_errors(c);
    if (r != RLC_OK) return r;
    DevOcc& o = c->occ;
    o.box = c->box;
    o.K = K;
    o.res = c->cfg.occ_grid_res;
    if (o.res) {
        float lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = hpart[a];
            hi[a] = hpart[3 * nb + a];
            for (uint32_t p = 1; p < nb; ++p) {
                lo[a] = std::min(lo[a], hpart[3 * p + a]);
                hi[a] = std::max(hi[a], hpart[3 * nb + 3 * p + a]);
            }
        }
        occ_grid_bounds(o, lo, hi, o.res);
        const uint32_t ncell = o.res * o.res * o.res;
        uint32_t *counts = nullptr, *start = nullptr, *cursor = nullptr, *scan_tmp = nullptr;
        r = dalloc(c, &counts, ncell);
        if (r == RLC_OK) r = dalloc(c, &start, (size_t)ncell + 1);
        if (r == RLC_OK) r = dalloc(c, &scan_tmp, scan_scratch_entries((size_t)ncell + 1) + 1);
        if (r == RLC_OK) r = dalloc(c, &cursor, ncell);
        if (r == RLC_OK) r = dalloc(c, &c->occ_head, ncell);
        hipError_t e = hipSuccess;
        auto step = [&](hipError_t x) {
            if (e == hipSuccess) e = x;
        };
        uint32_t total = 0;
        if (r == RLC_OK) {
            step(launch_fill_u32(counts, 0u, ncell, c->stream));
            step(launch_fill_u32(cursor, 0u, ncell, c->stream));
            step(launch_occ_count(c->box, K, o, counts, c->stream));
            step(launch_occ_sizes(counts, ncell, start, c->stream));
            step(launch_exclusive_scan(start, ncell + 1, scan_tmp, c->stream));
            step(hipMemcpyAsync(&total, start + ncell, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
            step(hipStreamSynchronize(c->stream));
        }
        if (r == RLC_OK && e == hipSuccess) {
            if (total >= RLC_OCC_PAYLOAD || K > RLC_OCC_PAYLOAD)
                r = fail(c, RLC_EINVAL, "too many occluder references for the grid (%u)", total);
            else
                r = dalloc(c, &c->occ_ref, total);
        }
        if (r == RLC_OK && e == hipSuccess) {
            o.head = c->occ_head;
            o.ref = c->occ_ref;
            step(launch_occ_lists(c->box, K, o, counts, start, cursor, c->occ_head, c->occ_ref, c->stream));
            step(launch_occ_skip(c->occ_head, counts, cursor, o.res, c->stream));
            step(hipStreamSynchronize(c->stream));
        }
        dfree(counts);
        dfree(start);
        dfree(cursor);
        dfree(scan_tmp);
        if (r != RLC_OK) return r;
        if (e != hipSuccess) return fail(c, RLC_EHIP, "occluder grid: %s", hipGetErrorString(e));
    }
    c->K = K;
    c->occ_set = true;
    return RLC_OK;
}

int rlc_sample(rlc_ctx* c, const float* d_pos, const float* d_nrm, uint32_t P, uint32_t spp, uint32_t frame,
               const rlc_samples* out) {
    RLC_TRY(check_frame_args(c, d_pos, P, spp));
    if (!out) return fail(c, RLC_EINVAL, "null sample records");
    if (P && !d_nrm && (c->cfg.normal_bits || c->cfg.jitter > 0.0f))
        return fail(c, RLC_EINVAL, "normals are needed for 5-D cells and jitter");
    RLC_HIP(c, launch_sample(frame_params(c), d_pos, d_nrm, P, spp, frame, *out, c->stream));
    return RLC_OK;
}

int rlc_shade(rlc_ctx* c, const float* d_pos, const float* d_nrm, uint32_t P, uint32_t spp,
              const rlc_samples* in, float* d_radiance, float* d_contrib, float* d_reward) {
    RLC_TRY(check_frame_args(c, d_pos, P, spp));
    if (!in || !d_nrm || !d_radiance || !in->d_light || !in->d_inv_pdf || !in->d_y || !in->d_slot)
        return fail(c, RLC_EINVAL, "missing shade input");
    if (c->cfg.reward_mode == 1 && (!in->d_cell || !in->d_ready))
        return fail(c, RLC_EINVAL, "cluster-size rewards need cell and ready records");
    RLC_HIP(c, launch_shade(frame_params(c), d_pos, d_nrm, P, spp, *in, d_radiance, d_contrib, d_reward, c->stream));
    return RLC_OK;
}

int rlc_learn(rlc_ctx* c, const rlc_samples* in, const float* d_reward, uint32_t n) {
    RLC_TRY(need_tree(c));
    if (n == 0) return RLC_OK;
    if (!in || !in->d_cell || !in->d_slot || !d_reward) return fail(c, RLC_EINVAL, "missing learn input");
    if (c->mix_cdf && !in->d_comp)
        return fail(c, RLC_EINVAL, "with the mixture on, learning needs the component records");
    RLC_HIP(c, launch_learn(frame_params(c), *in, d_reward, n, c->stream));
    return RLC_OK;
}

int rlc_adapt_cuts(rlc_ctx* c) {
    RLC_TRY(need_tree(c));
    RLC_HIP(c, launch_adapt(adapt_params(c), c->stream));
    return RLC_OK;
}

}  // extern "C"

namespace {

// One pass (the fused kernel, then the end of pass), arguments checked;
// with `timed`, HIP events around both kernels.
int frame_pass(rlc_ctx* c, const float* d_pos, const float* d_nrm, uint32_t P, uint32_t spp, uint32_t frame,
               float* d_radiance, bool timed) {
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (timed) {
        for (auto& e : ev) {
            e = take_event(c);
            if (!e) return fail(c, RLC_EHIP, "hipEventCreate failed");
        }
        RLC_HIP(c, hipEventRecord(ev[0], c->stream));
    }
    // the fused kernel's blocks run longest first when the pass before had
    // as many blocks (its durations ordered them); every pass records its
    // blocks' durations, and the end-of-pass launch orders them for the next
    const uint64_t nb = ((uint64_t)P * spp + RLC_FRAME_BLOCK - 1u) / RLC_FRAME_BLOCK;
    const bool sched = nb > 0 && nb <= RLC_ORDER_MAX_BLOCKS;
    FrameParams fp = frame_params(c);
    if (sched) {
        fp.blk_cost = c->blk_cost;
        fp.blk_order = c->blk_ordered == nb ? c->blk_order : nullptr;
    }
    RLC_HIP(c, launch_frame(fp, d_pos, d_nrm, P, spp, frame, d_radiance, c->stream));
    if (timed) RLC_HIP(c, hipEventRecord(ev[1], c->stream));
    AdaptParams ap = adapt_params(c);
    if (sched) {
        ap.blk_cost = c->blk_cost;
        ap.blk_order = c->blk_order;
        ap.blk_n = (uint32_t)nb;
    }
    RLC_HIP(c, launch_adapt(ap, c->stream));
    // (after a failed launch the order from an earlier pass stays, still a
    // permutation of its blocks)
    c->blk_ordered = sched ? (uint32_t)nb : 0u;
    if (timed) {
        RLC_HIP(c, hipEventRecord(ev[2], c->stream));
        for (auto& e : ev) c->pending.push_back(e);
    }
    return RLC_OK;
}

int check_sub_args(rlc_ctx* c, const float* d_pos, const float* d_nrm, uint32_t P, uint32_t spp, uint32_t n_sub,
                   uint32_t frame, const float* d_radiance) {
    RLC_TRY(check_frame_args(c, d_pos, P, spp));
    if (n_sub == 0 || spp % n_sub != 0) return fail(c, RLC_EINVAL, "spp (%u) is not a multiple of n_sub (%u)", spp, n_sub);
    if ((uint64_t)frame * n_sub + (n_sub - 1u) > 0xFFFFFFFFull)
        return fail(c, RLC_EINVAL, "pass index of frame %u x %u sub-frames exceeds 32 bits", frame, n_sub);
    if (P && (!d_nrm || !d_radiance)) return fail(c, RLC_EINVAL, "null normal or radiance array");
    return RLC_OK;
}

// The n_sub passes of one frame; passes after the first write their
// radiance to `buf` (P x 3 floats), which is then added to d_radiance.
int sub_passes(rlc_ctx* c, const float* d_pos, const float* d_nrm, uint32_t P, uint32_t spp, uint32_t n_sub,
               uint32_t frame, float* d_radiance, float* buf, bool timed) {
    const size_t n = (size_t)P * 3;
    const float scale = 1.0f / (float)n_sub;
    for (uint32_t j = 0; j < n_sub; ++j) {
        RLC_TRY(frame_pass(c, d_pos, d_nrm, P, spp / n_sub, frame * n_sub + j, j ? buf : d_radiance, timed));
        if (j) RLC_HIP(c, launch_accum(d_radiance, buf, n, scale, j + 1u == n_sub, c->stream));
    }
    return RLC_OK;
}

}  // namespace

extern "C" {

int rlc_frame(rlc_ctx* c, const float* d_pos, const float* d_nrm, uint32_t P, uint32_t spp, uint32_t frame,
              float* d_radiance) {
    RLC_TRY(check_frame_args(c, d_pos, P, spp));
    if (P && (!d_nrm || !d_radiance)) return fail(c, RLC_EINVAL, "null normal or radiance array");
    return frame_pass(c, d_pos, d_nrm, P, spp, frame, d_radiance, c->timing);
}

int rlc_frame_sub(rlc_ctx* c, const float* d_pos, const float* d_nrm, uint32_t P, uint32_t spp, uint32_t n_sub,
                  uint32_t frame, float* d_radiance) {
    RLC_TRY(check_sub_args(c, d_pos, d_nrm, P, spp, n_sub, frame, d_radiance));
    if (n_sub == 1) return rlc_frame(c, d_pos, d_nrm, P, spp, frame, d_radiance);
    if (P == 0) return RLC_OK;
    const size_t n = (size_t)P * 3;
    if (n > c->sub_cap) {
        // earlier passes may still read the old buffer
        RLC_HIP(c, hipStreamSynchronize(c->stream));
        dfree(c->sub_buf);
        c->sub_buf = nullptr;
        c->sub_cap = 0;
        RLC_TRY(dalloc(c, &c->sub_buf, n));
        c->sub_cap = n;
    }
    return sub_passes(c, d_pos, d_nrm, P, spp, n_sub, frame, d_radiance, c->sub_buf, c->timing);
}

int rlc_frame_sub_noalloc(rlc_ctx* c, const float* d_pos, const float* d_nrm, uint32_t P, uint32_t spp,
                          uint32_t n_sub, uint32_t frame, float* d_radiance) {
    RLC_TRY(check_sub_args(c, d_pos, d_nrm, P, spp, n_sub, frame, d_radiance));
    if (P > RLC_NOALLOC_MAX_POINTS)
        return fail(c, RLC_EINVAL, "%u points exceed the %u that rlc_frame_sub_noalloc's scratch holds", P,
                    RLC_NOALLOC_MAX_POINTS);
    if (!c->noalloc_scratch) return fail(c, RLC_ESTATE, "no scratch address for this device");
    if (P == 0) return RLC_OK;
    if (n_sub == 1) return frame_pass(c, d_pos, d_nrm, P, spp, frame, d_radiance, false);
    return sub_passes(c, d_pos, d_nrm, P, spp, n_sub, frame, d_radiance, c->noalloc_scratch, false);
}

int rlc_visible(rlc_ctx* c, const float* d_x, const float* d_y, uint32_t n, uint8_t* d_vis) {
    if (!c) return RLC_EINVAL;
    if (n == 0) return RLC_OK;
    if (!d_x || !d_y || !d_vis) return fail(c, RLC_EINVAL, "null array");
    DevOcc o = c->occ;
    o.K = c->occ_set ? c->K : 0u;
    RLC_HIP(c, launch_visible(o, c->cfg.t_lo, d_x, d_y, n, d_vis, c->stream));
    return RLC_OK;
}

int rlc_cell_keys(rlc_ctx* c, const float* d_pos, uint32_t n, uint64_t* d_keys) {
    if (!c) return RLC_EINVAL;
    if (n == 0) return RLC_OK;
    if (!d_pos || !d_keys) return fail(c, RLC_EINVAL, "null array");
    RLC_HIP(c, launch_cell_keys(frame_params(c), d_pos, n, d_keys, c->stream));
    return RLC_OK;
}

int rlc_image_error(rlc_ctx* c, const float* d_img, const float* d_ref, uint32_t n, double* h_out) {
    if (!c) return RLC_EINVAL;
    if (!h_out || (n && (!d_img || !d_ref))) return fail(c, RLC_EINVAL, "null array");
    if (n == 0) {
        for (int i = 0; i < 5; ++i) h_out[i] = 0.0;
        return RLC_OK;
    }
    uint32_t nb = std::min<uint32_t>(1024u, blocks_for(n));
    RLC_HIP(c, launch_image_error(d_img, d_ref, n, c->d_partial, nb, c->stream));
    std::vector<double> h(6 * (size_t)nb);
    RLC_HIP(c, hipMemcpyAsync(h.data(), c->d_partial, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
    RLC_HIP(c, hipStreamSynchronize(c->stream));
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t b = 0; b < nb; ++b) {
        for (int f = 0; f < 5; ++f) s[f] += h[6 * b + f];
        s[5] = std::max(s[5], h[6 * b + 5]);
    }
    double mean = s[0] / n;
    h_out[0] = mean;
    h_out[1] = std::max(0.0, s[1] / n - mean * mean);
    h_out[2] = s[2] / n;
    h_out[3] = s[4] > 0.0 ? s[3] / s[4] : 0.0;
    h_out[4] = s[5];
    return RLC_OK;
}

int rlc_sync(rlc_ctx* c) {
    if (!c) return RLC_EINVAL;
    RLC_HIP(c, hipStreamSynchronize(c->stream));
    return read_device_errors(c);
}

// The rows in use, stripe by stripe (a stripe's counter passes its rows
// once the stripe is full: the refused creations count too).
int rows_in_use(rlc_ctx* c, std::vector<uint32_t>* rows_out, uint32_t* h_n) {
    const DevCells& d = c->cells;
    std::vector<uint32_t> cnt((size_t)d.stripes * RLC_NLIVE_STRIDE);
    RLC_HIP(c, hipMemcpyAsync(cnt.data(), d.n_live, sizeof(uint32_t) * cnt.size(), hipMemcpyDeviceToHost, c->stream));
    RLC_HIP(c, hipStreamSynchronize(c->stream));
    uint32_t n = 0;
    for (uint32_t s = 0; s < d.stripes; ++s) {
        const uint32_t used = std::min(cnt[(size_t)s * RLC_NLIVE_STRIDE], d.stripe_rows);
        if (rows_out)
            for (uint32_t k = 0; k < used; ++k) rows_out->push_back(k * d.stripes + s);
        n += used;
    }
    *h_n = n;
    return RLC_OK;
}

int rlc_num_cells(rlc_ctx* c, uint32_t* h_n) {
    if (!c || !h_n) return RLC_EINVAL;
    return rows_in_use(c, nullptr, h_n);
}

int rlc_meff(rlc_ctx* c, uint32_t* h_meff) {
    RLC_TRY(need_tree(c));
    if (!h_meff) return RLC_EINVAL;
    *h_meff = c->Meff;
    return RLC_OK;
}

int rlc_dump_cells(rlc_ctx* c, uint32_t max_cells, uint64_t* h_keys, uint32_t* h_ready, uint32_t* h_node,
                   uint32_t* h_end, float* h_Q, float* h_Qt, float* h_C, uint64_t* h_sum, uint32_t* h_cnt) {
    RLC_TRY(need_tree(c));
    RLC_TRY(rlc_sync(c));
    uint32_t n = 0;
    std::vector<uint32_t> used;
    RLC_TRY(rows_in_use(c, &used, &n));
    if (n == 0) return RLC_OK;
    const DevCells& d = c->cells;
    // the rows in use hold the created cells; each row's slot holds its key
    std::vector<uint32_t> slot_of(d.rows), ready_all(d.rows), ready(n), order(n);
    std::vector<unsigned long long> words(d.capacity);
    RLC_HIP(c, hipMemcpy(slot_of.data(), d.live, sizeof(uint32_t) * d.rows, hipMemcpyDeviceToHost));
    RLC_HIP(c, hipMemcpy(ready_all.data(), d.ready, sizeof(uint32_t) * d.rows, hipMemcpyDeviceToHost));
    RLC_HIP(c, hipMemcpy(words.data(), d.keys, sizeof(unsigned long long) * d.capacity, hipMemcpyDeviceToHost));
    std::vector<uint64_t> key(n);
    for (uint32_t i = 0; i < n; ++i) {
        key[i] = ((uint64_t)c->cfg.scene_id << 32) | (words[slot_of[used[i]]] & 0xFFFFFFFFull);
        ready[i] = ready_all[used[i]];
        order[i] = used[i];
    }
    std::vector<uint32_t> idx(n);
    for (uint32_t i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return key[a] < key[b]; });
    {
        std::vector<uint64_t> k2(n);
        std::vector<uint32_t> r2(n), o2(n);
        for (uint32_t i = 0; i < n; ++i) {
            k2[i] = key[idx[i]];
            r2[i] = ready[idx[i]];
            o2[i] = order[idx[i]];
        }
        key.swap(k2);
        ready.swap(r2);
        order.swap(o2);
    }
    uint32_t rows = std::min(n, max_cells);
    if (rows == 0) return RLC_OK;
    for (uint32_t i = 0; i < rows; ++i) {
        if (h_keys) h_keys[i] = key[i];
        if (h_ready) h_ready[i] = ready[i];
    }
    const uint32_t Meff = c->Meff;
    size_t cnt = (size_t)rows * Meff;
    uint32_t* d_rows = nullptr;
    uint32_t *dn = nullptr, *de = nullptr, *dc = nullptr;
    float *dq = nullptr, *dqt = nullptr, *dC = nullptr;
    unsigned long long* ds = nullptr;
    int r = dalloc(c, &d_rows, rows);
    if (r == RLC_OK && h_node) r = dalloc(c, &dn, cnt);
    if (r == RLC_OK && h_end) r = dalloc(c, &de, cnt);
    if (r == RLC_OK && h_Q) r = dalloc(c, &dq, cnt);
    if (r == RLC_OK && h_Qt) r = dalloc(c, &dqt, cnt);
    if (r == RLC_OK && h_C) r = dalloc(c, &dC, cnt);
    if (r == RLC_OK && h_sum) r = dalloc(c, &ds, cnt);
    if (r == RLC_OK && h_cnt) r = dalloc(c, &dc, cnt);
    hipError_t e = hipSuccess;
    if (r == RLC_OK) {
        e = hipMemcpy(d_rows, order.data(), sizeof(uint32_t) * rows, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = launch_gather_cells(d, Meff, d_rows, rows, dn, de, dq, dqt, dC, ds, dc, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess && h_node) e = hipMemcpy(h_node, dn, sizeof(uint32_t) * cnt, hipMemcpyDeviceToHost);
        if (e == hipSuccess && h_end) e = hipMemcpy(h_end, de, sizeof(uint32_t) * cnt, hipMemcpyDeviceToHost);
        if (e == hipSuccess && h_Q) e = hipMemcpy(h_Q, dq, sizeof(float) * cnt, hipMemcpyDeviceToHost);
        if (e == hipSuccess && h_Qt) e = hipMemcpy(h_Qt, dqt, sizeof(float) * cnt, hipMemcpyDeviceToHost);
        if (e == hipSuccess && h_C) e = hipMemcpy(h_C, dC, sizeof(float) * cnt, hipMemcpyDeviceToHost);
        if (e == hipSuccess && h_sum) e = hipMemcpy(h_sum, ds, sizeof(uint64_t) * cnt, hipMemcpyDeviceToHost);
        if (e == hipSuccess && h_cnt) e = hipMemcpy(h_cnt, dc, sizeof(uint32_t) * cnt, hipMemcpyDeviceToHost);
    }
    dfree(d_rows);
    dfree(dn);
    dfree(de);
    dfree(dq);
    dfree(dqt);
    dfree(dC);
    dfree(ds);
    dfree(dc);
    if (r != RLC_OK) return r;
    if (e != hipSuccess) return fail(c, RLC_EHIP, "dump: %s", hipGetErrorString(e));
    return RLC_OK;
}

int rlc_load_cells(rlc_ctx* c, uint32_t n, const uint64_t* h_keys, const uint32_t* h_node, const float* h_Q) {
    RLC_TRY(need_tree(c));
    if (n == 0) return RLC_OK;
    if (!h_keys || !h_node || !h_Q) return fail(c, RLC_EINVAL, "null array");
    RLC_TRY(rlc_sync(c));
    const uint32_t N = c->N, Meff = c->Meff, nn = 2u * N - 1u;
    std::vector<uint32_t> first(nn), last(nn);
    RLC_HIP(c, hipMemcpy(first.data(), c->first, sizeof(uint32_t) * nn, hipMemcpyDeviceToHost));
    RLC_HIP(c, hipMemcpy(last.data(), c->last, sizeof(uint32_t) * nn, hipMemcpyDeviceToHost));
    std::vector<uint64_t> sorted(h_keys, h_keys + n);
    std::sort(sorted.begin(), sorted.end());
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t key = sorted[i];
        if ((key >> 32) != (uint64_t)c->cfg.scene_id || (key & 0xFFFFFFFFull) >= c->cell_index_limit)
            return fail(c, RLC_EINVAL, "cell key %llu is not a cell of this scene", (unsigned long long)key);
        if (i && key == sorted[i - 1]) return fail(c, RLC_EINVAL, "cell key %llu given twice", (unsigned long long)key);
    }
    if (n > c->cells.stripes * c->cells.stripe_rows)
        return fail(c, RLC_EINVAL, "more cells than the table holds rows for (%u)",
                    c->cells.stripes * c->cells.stripe_rows);
    for (uint32_t i = 0; i < n; ++i) {
        // the cut partitions the lights in range order: each node starts
        // right after the previous one ends, the first at 0, the last at N-1
        uint32_t next = 0;
        for (uint32_t s = 0; s < Meff; ++s) {
            const uint32_t nd = h_node[(size_t)i * Meff + s];
            const float q = h_Q[(size_t)i * Meff + s];
            if (nd >= nn || first[nd] != next)
                return fail(c, RLC_EINVAL, "cell %u: the cut is not a partition of the lights at slot %u", i, s);
            if (!(q >= 0.0f && q <= 3.402823466e38f))
                return fail(c, RLC_EINVAL, "cell %u: Q[%u] is negative or not finite", i, s);
            next = last[nd] + 1u;
        }
        if (next != N) return fail(c, RLC_EINVAL, "cell %u: the cut does not cover every light", i);
    }
    unsigned long long* dk = nullptr;
    uint32_t* dn = nullptr;
    float* dq = nullptr;
    const size_t cnt = (size_t)n * Meff;
    int r = dalloc(c, &dk, n);
    if (r == RLC_OK) r = dalloc(c, &dn, cnt);
    if (r == RLC_OK) r = dalloc(c, &dq, cnt);
    hipError_t e = hipSuccess;
    if (r == RLC_OK) {
        e = hipMemcpyAsync(dk, h_keys, sizeof(uint64_t) * n, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(dn, h_node, sizeof(uint32_t) * cnt, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(dq, h_Q, sizeof(float) * cnt, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = launch_load_cells(adapt_params(c), dk, dn, dq, n, c->d_err, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    dfree(dk);
    dfree(dn);
    dfree(dq);
    if (r != RLC_OK) return r;
    if (e != hipSuccess) return fail(c, RLC_EHIP, "load cells: %s", hipGetErrorString(e));
    return read_device_errors(c);
}

int rlc_get_light_order(rlc_ctx* c, uint32_t* d_perm) {
    RLC_TRY(need_tree(c));
    if (!d_perm) return fail(c, RLC_EINVAL, "null array");
    RLC_HIP(c, hipMemcpyAsync(d_perm, c->perm, sizeof(uint32_t) * c->N, hipMemcpyDeviceToDevice, c->stream));
    return RLC_OK;
}

int rlc_dump_tree(rlc_ctx* c, uint32_t* h_perm, uint32_t* h_left, uint32_t* h_right, uint32_t* h_parent,
                  uint32_t* h_first, uint32_t* h_last, float* h_rec) {
    RLC_TRY(need_tree(c));
    RLC_HIP(c, hipStreamSynchronize(c->stream));
    const uint32_t N = c->N, nn = 2 * N - 1;
    if (h_perm) RLC_HIP(c, hipMemcpy(h_perm, c->perm, sizeof(uint32_t) * N, hipMemcpyDeviceToHost));
    if (h_left && N > 1) RLC_HIP(c, hipMemcpy(h_left, c->left, sizeof(uint32_t) * (N - 1), hipMemcpyDeviceToHost));
    if (h_right && N > 1) RLC_HIP(c, hipMemcpy(h_right, c->right, sizeof(uint32_t) * (N - 1), hipMemcpyDeviceToHost));
    if (h_parent) RLC_HIP(c, hipMemcpy(h_parent, c->parent, sizeof(uint32_t) * nn, hipMemcpyDeviceToHost));
    if (h_first) RLC_HIP(c, hipMemcpy(h_first, c->first, sizeof(uint32_t) * nn, hipMemcpyDeviceToHost));
    if (h_last) RLC_HIP(c, hipMemcpy(h_last, c->last, sizeof(uint32_t) * nn, hipMemcpyDeviceToHost));
    if (h_rec) RLC_HIP(c, hipMemcpy(h_rec, c->rec, sizeof(float4) * 4 * (size_t)N, hipMemcpyDeviceToHost));
    return RLC_OK;
}

int rlc_get_template(rlc_ctx* c, uint32_t* h_node, uint32_t* h_end, uint32_t* h_meff) {
    RLC_TRY(need_tree(c));
    RLC_HIP(c, hipStreamSynchronize(c->stream));
    if (h_node) RLC_HIP(c, hipMemcpy(h_node, c->tmpl_node, sizeof(uint32_t) * c->Meff, hipMemcpyDeviceToHost));
    if (h_end) RLC_HIP(c, hipMemcpy(h_end, c->tmpl_end, sizeof(uint32_t) * c->Meff, hipMemcpyDeviceToHost));
    if (h_meff) *h_meff = c->Meff;
    return RLC_OK;
}

int rlc_mlp_fixed_cut(rlc_ctx* c, uint32_t* h_node, uint32_t* h_end, uint32_t* h_m) {
    RLC_TRY(need_tree(c));
    RLC_HIP(c, hipStreamSynchronize(c->stream));
    if (h_node) RLC_HIP(c, hipMemcpy(h_node, c->fix_node, sizeof(uint32_t) * c->fix_M, hipMemcpyDeviceToHost));
    if (h_end) RLC_HIP(c, hipMemcpy(h_end, c->fix_end, sizeof(uint32_t) * c->fix_M, hipMemcpyDeviceToHost));
    if (h_m) *h_m = c->fix_M;
    return RLC_OK;
}

int rlc_mlp_init(rlc_ctx* c, uint64_t seed) {
    if (!c) return RLC_EINVAL;
    RLC_TRY(mlp_alloc(c));
    RLC_HIP(c, launch_mlp_init(c->mlp_master, c->cfg.scene_id, (uint32_t)(seed & 0xFFFFFFFFull),
                               (uint32_t)(seed >> 32), c->stream));
    return mlp_reset_optimizer(c);
}

int rlc_mlp_set_params(rlc_ctx* c, const float* d_params) {
    if (!c) return RLC_EINVAL;
    if (!d_params) return fail(c, RLC_EINVAL, "null parameter array");
    RLC_TRY(mlp_alloc(c));
    RLC_HIP(c, hipMemcpyAsync(c->mlp_master, d_params, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice,
                              c->stream));
    RLC_HIP(c, launch_fill_u32(c->d_err, 0u, 1, c->stream));
    RLC_HIP(c, launch_check_finite(c->mlp_master, kMlpParams, c->d_err, c->stream));
    RLC_TRY(read_device_errors(c));
    return mlp_reset_optimizer(c);
}

int rlc_mlp_copy_params(rlc_ctx* dst, rlc_ctx* src) {
    if (!dst || !src) return RLC_EINVAL;
    if (dst == src) return fail(dst, RLC_EINVAL, "a context takes weights from another context");
    if (!src->mlp_ready) return fail(dst, RLC_ESTATE, "the source network has no weights");
    RLC_TRY(mlp_alloc(dst));
    if (src->stream != dst->stream) {
        // dst's stream waits for the work enqueued so far on src's
        if (!src->join) RLC_HIP(dst, hipEventCreateWithFlags(&src->join, hipEventDisableTiming));
        RLC_HIP(dst, hipEventRecord(src->join, src->stream));
        RLC_HIP(dst, hipStreamWaitEvent(dst->stream, src->join, 0));
    }
    RLC_HIP(dst, hipMemcpyAsync(dst->mlp_master, src->mlp_master, sizeof(float) * kMlpParams,
                                hipMemcpyDeviceToDevice, dst->stream));
    return mlp_reset_optimizer(dst);
}

int rlc_mlp_get_params(rlc_ctx* c, float* d_params) {
    if (!c) return RLC_EINVAL;
    if (!c->mlp_ready) return fail(c, RLC_ESTATE, "the network has no weights");
    if (!d_params) return fail(c, RLC_EINVAL, "null parameter array");
    RLC_HIP(c, hipMemcpyAsync(d_params, c->mlp_master, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice,
                              c->stream));
    return RLC_OK;
}

int rlc_mlp_forward(rlc_ctx* c, const float* d_pos, const float* d_nrm, uint32_t P, float* d_cdf,
                    float* d_logits) {
    if (!c) return RLC_EINVAL;
    if (!c->mlp_ready) return fail(c, RLC_ESTATE, "the network has no weights");
    if (P == 0) return RLC_OK;
    if (!d_pos || !d_nrm) return fail(c, RLC_EINVAL, "null point array");
    if (!d_cdf && !d_logits) return fail(c, RLC_EINVAL, "no output");
    RLC_HIP(c, launch_mlp_forward(c->mlp_frag, c->mlp_master, mlp_encode_params(c), d_pos, d_nrm, P, d_cdf, d_logits,
                                  c->stream));
    return RLC_OK;
}

int rlc_mlp_grad(rlc_ctx* c, const float* d_pos, const float* d_nrm, uint32_t P, const uint32_t* d_pid,
                 const uint32_t* d_node, const float* d_w, uint32_t n, float* d_grad, float* h_loss) {
    if (!c) return RLC_EINVAL;
    RLC_TRY(check_tuples(c, d_pos, d_nrm, P, d_pid, d_node, d_w, n));
    if (!d_grad) return fail(c, RLC_EINVAL, "null gradient array");
    const uint32_t nb = std::max<uint32_t>(1u, (n + kMlpTuplesPerBlock - 1u) / kMlpTuplesPerBlock);
    RLC_TRY(mlp_partials(c, nb));
    RLC_HIP(c, launch_fill_u32(c->d_err, 0u, 1, c->stream));
    if (n == 0) {
        RLC_HIP(c, hipMemsetAsync(c->mlp_part_w, 0, sizeof(float), c->stream));
        RLC_HIP(c, hipMemsetAsync(c->mlp_part_loss, 0, sizeof(float), c->stream));
        RLC_HIP(c, hipMemsetAsync(c->mlp_partial, 0, sizeof(float) * kMlpParams, c->stream));
    }
    const uint16_t* xenc = nullptr;
    if (n) RLC_TRY(mlp_encoded_inputs(c, d_pos, d_nrm, P, &xenc));
    const MlpOrder identity{};
    RLC_HIP(c, launch_mlp_fwd_bwd(c->mlp_frag, c->mlp_master, mlp_encode_params(c), d_pos, d_nrm, P, xenc, identity,
                                  0u, d_pid, d_node, d_w, n, c->mlp_partial, c->mlp_part_w, c->mlp_part_loss,
                                  c->d_err, c->stream));
    RLC_HIP(c, launch_mlp_reduce(c->mlp_partial, c->mlp_part_w, c->mlp_part_loss, nb, 0u, d_grad, nullptr, nullptr,
                                 nullptr, nullptr, 0.0f, 0.0f, 0.0f, 0.0f, 1.0f, 1.0f, c->mlp_loss, c->stream));
    float loss = 0.0f;
    RLC_HIP(c, hipMemcpyAsync(&loss, c->mlp_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    RLC_TRY(read_device_errors(c));
    if (h_loss) *h_loss = loss;
    return RLC_OK;
}

int rlc_mlp_train(rlc_ctx* c, const float* d_pos, const float* d_nrm, uint32_t P, const uint32_t* d_pid,
                  const uint32_t* d_node, const float* d_w, uint32_t n, uint32_t epochs, uint32_t batch, float lr,
                  float* h_loss) {
    if (!c) return RLC_EINVAL;
    RLC_TRY(check_tuples(c, d_pos, d_nrm, P, d_pid, d_node, d_w, n));
    if (batch == 0 || batch > (1u << 24)) return fail(c, RLC_EINVAL, "batch must be in 1..2^24");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(c, RLC_EINVAL, "learning rate must be positive");
    if (n == 0 || epochs == 0) return RLC_OK;
    const uint32_t bmax = std::min(batch, n);
    const uint32_t nb = (bmax + kMlpTuplesPerBlock - 1u) / kMlpTuplesPerBlock;
    RLC_TRY(mlp_partials(c, nb));
    RLC_HIP(c, launch_fill_u32(c->d_err, 0u, 1, c->stream));
    const MlpEncode enc = mlp_encode_params(c);
    const uint16_t* xenc = nullptr;
    RLC_TRY(mlp_encoded_inputs(c, d_pos, d_nrm, P, &xenc));
    // a training step's two launches, with HIP events around and between
    // them while timing is on
    auto timed = [&](auto&& launch) -> int {
        hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
        if (c->timing) {
            for (auto& x : ev) {
                x = take_event(c);
                if (!x) return fail(c, RLC_EHIP, "hipEventCreate failed");
            }
            RLC_HIP(c, hipEventRecord(ev[0], c->stream));
        }
        RLC_TRY(launch(ev[1]));
        if (c->timing) {
            RLC_HIP(c, hipEventRecord(ev[2], c->stream));
            for (auto& x : ev) c->mlp_pending.push_back(x);
        }
        return RLC_OK;
    };
    for (uint32_t e = 0; e < epochs; ++e) {
        const MlpOrder ord = mlp_epoch_order(n, e, c->cfg.scene_id, c->cfg.seed);
        for (uint32_t b0 = 0; b0 < n; b0 += batch) {
            const uint32_t nbat = std::min(batch, n - b0);
            const uint32_t blocks = (nbat + kMlpTuplesPerBlock - 1u) / kMlpTuplesPerBlock;
            c->mlp_step += 1u;
            c->mlp_b1t *= (double)kAdamBeta1;
            c->mlp_b2t *= (double)kAdamBeta2;
            const float c1 = (float)(1.0 - c->mlp_b1t);
            const float c2 = (float)(1.0 - c->mlp_b2t);
            RLC_TRY(timed(
                [&](hipEvent_t mid) -> int {
                    RLC_HIP(c, launch_mlp_fwd_bwd(c->mlp_frag, c->mlp_master, enc, d_pos, d_nrm, P, xenc, ord, b0,
                                                  d_pid, d_node, d_w, nbat, c->mlp_partial, c->mlp_part_w,
                                                  c->mlp_part_loss, c->d_err, c->stream));
                    if (c->timing) RLC_HIP(c, hipEventRecord(mid, c->stream));
                    RLC_HIP(c, launch_mlp_reduce(c->mlp_partial, c->mlp_part_w, c->mlp_part_loss, blocks, 1u,
                                                 nullptr, c->mlp_master, c->mlp_m, c->mlp_v, c->mlp_frag, lr,
                                                 kAdamBeta1, kAdamBeta2, kAdamEps, c1, c2, c->mlp_loss,
                                                 c->stream));
                    return RLC_OK;
                }));
        }
    }
    if (!h_loss) return RLC_OK;  // asynchronous: bad tuples are reported by the next synchronising call
    float loss = 0.0f;
    RLC_HIP(c, hipMemcpyAsync(&loss, c->mlp_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    RLC_TRY(read_device_errors(c));
    *h_loss = loss;
    return RLC_OK;
}

int rlc_mlp_order(rlc_ctx* c, uint32_t n, uint32_t epoch, uint32_t* d_order) {
    if (!c) return RLC_EINVAL;
    if (n == 0) return RLC_OK;
    if (!d_order) return fail(c, RLC_EINVAL, "null array");
    RLC_HIP(c, launch_mlp_order(mlp_epoch_order(n, epoch, c->cfg.scene_id, c->cfg.seed), d_order, c->stream));
    return RLC_OK;
}

int rlc_set_mixture(rlc_ctx* c, const float* d_cdf, uint32_t rows, float w) {
    RLC_TRY(need_tree(c));
    if (!d_cdf) {
        c->mix_cdf = nullptr;
        c->mix_rows = 0;
        return RLC_OK;
    }
    if (rows == 0) return fail(c, RLC_EINVAL, "the mixture cdf has no rows");
    if (!(w >= 0.0f && w < 1.0f))
        return fail(c, RLC_EINVAL, "the network's share w must be in [0, 1): alone it may give a light density 0");
    if (w == 0.0f) {
        // the tabular method alone
        c->mix_cdf = nullptr;
        c->mix_rows = 0;
        return RLC_OK;
    }
    c->mix_cdf = d_cdf;
    c->mix_rows = rows;
    c->mix_w = w;
    return RLC_OK;
}

int rlc_set_footprints(rlc_ctx* c, const float* d_fp, uint32_t rows) {
    if (!c) return RLC_EINVAL;
    if (d_fp && rows) {
        RLC_HIP(c, launch_fill_u32(c->d_err, 0u, 1, c->stream));
        RLC_HIP(c, launch_check_nonneg(d_fp, rows, c->d_err, c->stream));
        RLC_HIP(c, hipStreamSynchronize(c->stream));
        const int r = read_device_errors(c);
        if (r != RLC_OK) return fail(c, r, "footprints must be finite and >= 0");
    }
    // batches over this context capture their parameters again
    c->generation += 1u;
    c->fp_arr = (d_fp && rows) ? d_fp : nullptr;
    c->fp_rows = c->fp_arr ? rows : 0u;
    return RLC_OK;
}

int rlc_set_sample_log(rlc_ctx* c, uint32_t* d_pid, uint32_t* d_node, float* d_w, uint64_t capacity) {
    if (!c) return RLC_EINVAL;
    if (!d_pid && !d_node && !d_w) {
        c->log_pid = nullptr;
        c->log_node = nullptr;
        c->log_w = nullptr;
        c->log_cap = 0;
        return RLC_OK;
    }
    if (!d_pid || !d_node || !d_w) return fail(c, RLC_EINVAL, "the sample log needs all three arrays");
    c->log_pid = d_pid;
    c->log_node = d_node;
    c->log_w = d_w;
    c->log_cap = capacity;
    return RLC_OK;
}

int rlc_set_timing(rlc_ctx* c, int enable) {
    if (!c) return RLC_EINVAL;
    c->timing = enable != 0;
    return RLC_OK;
}

int rlc_get_timing(rlc_ctx* c, double* h_ms_fused, double* h_ms_adapt, uint32_t* h_frames) {
    if (!c) return RLC_EINVAL;
    double f = 0.0, a = 0.0;
    uint32_t frames = (uint32_t)(c->pending.size() / 3);
    for (uint32_t i = 0; i < frames; ++i) {
        hipEvent_t* e = &c->pending[3 * i];
        RLC_HIP(c, hipEventSynchronize(e[2]));
        float t01 = 0.0f, t12 = 0.0f;
        RLC_HIP(c, hipEventElapsedTime(&t01, e[0], e[1]));
        RLC_HIP(c, hipEventElapsedTime(&t12, e[1], e[2]));
        f += t01;
        a += t12;
    }
    for (hipEvent_t e : c->pending) c->spare.push_back(e);
    c->pending.clear();
    if (h_ms_fused) *h_ms_fused = f;
    if (h_ms_adapt) *h_ms_adapt = a;
    if (h_frames) *h_frames = frames;
    return RLC_OK;
}

int rlc_get_mlp_timing(rlc_ctx* c, double* h_ms_fwd_bwd, double* h_ms_update, uint32_t* h_steps) {
    if (!c) return RLC_EINVAL;
    double f = 0.0, u = 0.0;
    uint32_t steps = (uint32_t)(c->mlp_pending.size() / 3);
    for (uint32_t i = 0; i < steps; ++i) {
        hipEvent_t* e = &c->mlp_pending[3 * i];
        RLC_HIP(c, hipEventSynchronize(e[2]));
        float t01 = 0.0f, t12 = 0.0f;
        RLC_HIP(c, hipEventElapsedTime(&t01, e[0], e[1]));
        RLC_HIP(c, hipEventElapsedTime(&t12, e[1], e[2]));
        f += t01;
        u += t12;
    }
    for (hipEvent_t e : c->mlp_pending) c->spare.push_back(e);
    c->mlp_pending.clear();
    if (h_ms_fwd_bwd) *h_ms_fwd_bwd = f;
    if (h_ms_update) *h_ms_update = u;
    if (h_steps) *h_steps = steps;
    return RLC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched passes
// ---------------------------------------------------------------------------
struct rlc_batch {
    std::vector<rlc_batch_scene> scenes;
    hipStream_t stream = nullptr;
    rlc_schedule sched{512, 8, 1, 0};
    uint32_t n_cu = 256;
    uint32_t total_items = 0;
    BatchScene* d_scenes = nullptr;
    AdaptParams* d_adapt = nullptr;
    uint32_t* d_counter = nullptr;
    uint32_t* d_frame = nullptr;
    std::vector<uint32_t*> perms;  // cell-order visiting permutation per scene
    std::vector<uint32_t> gens;    // each context's generation when the graph was captured
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t next_frame = 0;
    bool frame_known = false;
};

namespace {

void batch_drop_graph(rlc_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Visiting order of a scene's points sorted by cell (stable: ties keep
// input order), built once with the library's radix sort.
int batch_make_perm(rlc_ctx* c, const rlc_batch_scene& sc, uint32_t** out) {
    *out = nullptr;
    uint32_t *lin = nullptr, *idx = nullptr, *kt = nullptr, *vt = nullptr, *hist = nullptr;
    int r = dalloc(c, &lin, sc.P);
    if (r == RLC_OK) r = dalloc(c, &idx, sc.P);
    if (r == RLC_OK) r = dalloc(c, &kt, sc.P);
    if (r == RLC_OK) r = dalloc(c, &vt, sc.P);
    if (r == RLC_OK) r = dalloc(c, &hist, radix_sort_hist_entries(sc.P));
    hipError_t e = hipSuccess;
    if (r == RLC_OK) {
        uint64_t cells = (uint64_t)c->cfg.grid_dims[0] * c->cfg.grid_dims[1] * c->cfg.grid_dims[2];
        int bits = 1;
        while (bits < 32 && (1ull << bits) < cells) ++bits;
        e = launch_cell_lin(frame_params(c), sc.d_pos, sc.P, lin, idx, c->stream);
        if (e == hipSuccess) e = radix_sort_pairs(lin, idx, kt, vt, hist, sc.P, bits, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    dfree(lin);
    dfree(kt);
    dfree(vt);
    dfree(hist);
    if (r != RLC_OK || e != hipSuccess) {
        dfree(idx);
        return r != RLC_OK ? r : fail(c, RLC_EHIP, "cell order: %s", hipGetErrorString(e));
    }
    *out = idx;
    return RLC_OK;
}

int batch_upload(rlc_batch* b) {
    rlc_ctx* c0 = b->scenes[0].ctx;
    const uint32_t tile = b->sched.tile;
    std::vector<BatchScene> hs(b->scenes.size());
    std::vector<AdaptParams> ha(b->scenes.size());
    uint32_t item = 0;
    for (size_t i = 0; i < b->scenes.size(); ++i) {
        const rlc_batch_scene& sc = b->scenes[i];
        BatchScene& d = hs[i];
        d.fp = frame_params(sc.ctx);
        // batched passes draw from the cells' cuts alone and keep no log
        d.fp.mix_cdf = nullptr;
        d.fp.log_pid = nullptr;
        d.fp.log_node = nullptr;
        d.fp.log_w = nullptr;
        d.pos = sc.d_pos;
        d.nrm = sc.d_nrm;
        d.perm = b->sched.cell_sorted ? b->perms[i] : nullptr;
        d.radiance = sc.d_radiance;
        d.P = sc.P;
        d.spp = sc.spp;
        uint64_t n = (uint64_t)sc.P * sc.spp;
        d.items = (uint32_t)((n + tile - 1) / tile);
        d.item_begin = item;
        item += d.items;
        ha[i] = adapt_params(sc.ctx);
    }
    b->total_items = item;
    // the previous graph may still read the tables
    RLC_HIP(c0, hipStreamSynchronize(b->stream));
    RLC_HIP(c0, hipMemcpy(b->d_scenes, hs.data(), sizeof(BatchScene) * hs.size(), hipMemcpyHostToDevice));
    RLC_HIP(c0, hipMemcpy(b->d_adapt, ha.data(), sizeof(AdaptParams) * ha.size(), hipMemcpyHostToDevice));
    b->gens.resize(b->scenes.size());
    for (size_t i = 0; i < b->scenes.size(); ++i) b->gens[i] = b->scenes[i].ctx->generation;
    return RLC_OK;
}

// Capture one pass (reset the work counter, the persistent frame kernel, the
// adapt kernel over every scene, advance the device frame index).
int batch_capture(rlc_batch* b) {
    rlc_ctx* c0 = b->scenes[0].ctx;
    batch_drop_graph(b);
    RLC_TRY(batch_upload(b));
    const uint32_t grid = b->sched.blocks_per_cu * b->n_cu;
    const uint32_t rounds = b->sched.tile / 256u;
    RLC_HIP(c0, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_batch_begin(b->d_counter, b->stream);
    if (e == hipSuccess)
        e = launch_batch_frame(b->d_scenes, (uint32_t)b->scenes.size(), b->total_items, rounds, b->sched.dynamic,
                               grid, b->d_counter, b->d_frame, b->stream);
    uint32_t meff_max = 1, steps_max = 0;
    for (const auto& sc : b->scenes) {
        meff_max = std::max(meff_max, sc.ctx->Meff);
        steps_max = std::max(steps_max, sc.ctx->cfg.split_steps);
    }
    // up to 16 scenes whose cuts have up to 64 clusters, one split-collapse
    // step: 16 cells per block over all scenes' rows in use (as k_adapt16
    // does for one scene); otherwise one wave per cell, scene after scene
    if (e == hipSuccess && meff_max <= 64u && steps_max <= 1u && b->scenes.size() <= 16u)
        e = launch_batch_adapt16(b->d_adapt, (uint32_t)b->scenes.size(), b->stream);
    else if (e == hipSuccess)
        e = launch_batch_adapt(b->d_adapt, (uint32_t)b->scenes.size(), meff_max, b->stream);
    if (e == hipSuccess) e = launch_batch_end(b->d_frame, b->stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(c0, RLC_EHIP, "batch graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = g;
    RLC_HIP(c0, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return RLC_OK;
}

bool valid_schedule(const rlc_schedule& s) {
    return s.tile >= 256 && s.tile % 256 == 0 && s.tile <= 65536 && s.blocks_per_cu >= 1 && s.blocks_per_cu <= 64 &&
           s.dynamic <= 1 && s.cell_sorted <= 1;
}

}  // namespace

extern "C" {

int rlc_batch_create(const rlc_batch_scene* scenes, uint32_t n, void* stream, rlc_batch** out) {
    if (!out) return RLC_EINVAL;
    *out = nullptr;
    if (!scenes || n == 0) return RLC_EINVAL;
    if (!stream) return fail(scenes[0].ctx, RLC_EINVAL, "a batch needs a non-default stream (graph capture)");
    for (uint32_t i = 0; i < n; ++i) {
        const rlc_batch_scene& sc = scenes[i];
        if (!sc.ctx) return RLC_EINVAL;
        if (!sc.ctx->tree_built) return fail(sc.ctx, RLC_ESTATE, "batch scene %u: the light tree has not been built", i);
        if (sc.ctx->stream != (hipStream_t)stream)
            return fail(sc.ctx, RLC_EINVAL, "batch scene %u: its context uses another stream", i);
        if (sc.P && (!sc.d_pos || !sc.d_nrm || !sc.d_radiance))
            return fail(sc.ctx, RLC_EINVAL, "batch scene %u: null array", i);
        if (sc.spp == 0 || sc.spp > 64 || (sc.spp & (sc.spp - 1)))
            return fail(sc.ctx, RLC_EINVAL, "batch scene %u: spp must be a power of two <= 64", i);
        if ((uint64_t)sc.P * sc.spp > 0xFFFFFFFFull) return fail(sc.ctx, RLC_EINVAL, "batch scene %u too large", i);
        for (uint32_t j = 0; j < i; ++j)
            if (scenes[j].ctx == sc.ctx) return fail(sc.ctx, RLC_EINVAL, "a context appears twice in the batch");
    }
    rlc_batch* b = new (std::nothrow) rlc_batch();
    if (!b) return RLC_ENOMEM;
    b->scenes.assign(scenes, scenes + n);
    b->stream = (hipStream_t)stream;
    rlc_ctx* c0 = scenes[0].ctx;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
        b->n_cu = (uint32_t)prop.multiProcessorCount;
    int r = dalloc(c0, &b->d_scenes, n);
    if (r == RLC_OK) r = dalloc(c0, &b->d_adapt, n);
    if (r == RLC_OK) r = dalloc(c0, &b->d_counter, 1);
    if (r == RLC_OK) r = dalloc(c0, &b->d_frame, 1);
    b->perms.assign(n, nullptr);
    for (uint32_t i = 0; r == RLC_OK && i < n; ++i)
        if (scenes[i].P) r = batch_make_perm(scenes[i].ctx, scenes[i], &b->perms[i]);
    if (r == RLC_OK) {
        hipError_t e = launch_set_u32(b->d_frame, 0u, b->stream);
        if (e != hipSuccess) r = fail(c0, RLC_EHIP, "batch: %s", hipGetErrorString(e));
    }
    if (r == RLC_OK) r = batch_capture(b);
    for (uint32_t i = 0; i < n; ++i) scenes[i].ctx->batch_refs += 1u;
    if (r != RLC_OK) {
        rlc_batch_destroy(b);
        return r;
    }
    *out = b;
    return RLC_OK;
}

int rlc_batch_destroy(rlc_batch* b) {
    if (!b) return RLC_OK;
    (void)hipStreamSynchronize(b->stream);
    for (auto& sc : b->scenes) sc.ctx->batch_refs -= 1u;
    batch_drop_graph(b);
    dfree(b->d_scenes);
    dfree(b->d_adapt);
    dfree(b->d_counter);
    dfree(b->d_frame);
    for (auto& p : b->perms) dfree(p);
    delete b;
    return RLC_OK;
}

int rlc_batch_set_schedule(rlc_batch* b, const rlc_schedule* sched) {
    if (!b || !sched) return RLC_EINVAL;
    if (!valid_schedule(*sched)) return fail(b->scenes[0].ctx, RLC_EINVAL, "invalid schedule");
    RLC_HIP(b->scenes[0].ctx, hipStreamSynchronize(b->stream));
    b->sched = *sched;
    return batch_capture(b);
}

int rlc_batch_get_schedule(rlc_batch* b, rlc_schedule* sched) {
    if (!b || !sched) return RLC_EINVAL;
    *sched = b->sched;
    return RLC_OK;
}

int rlc_batch_frame(rlc_batch* b, uint32_t frame) {
    if (!b) return RLC_EINVAL;
    rlc_ctx* c0 = b->scenes[0].ctx;
    // a scene's tree or occluders were rebuilt since the capture: the graph
    // holds freed addresses, so capture again from the current buffers
    bool stale = false;
    for (size_t i = 0; i < b->scenes.size(); ++i) {
        const rlc_ctx* c = b->scenes[i].ctx;
        if (c->generation != b->gens[i]) stale = true;
        if (!c->tree_built) return fail(b->scenes[i].ctx, RLC_ESTATE, "batch scene %zu has no light tree", i);
    }
    if (stale) RLC_TRY(batch_capture(b));
    if (!b->frame_known || frame != b->next_frame) RLC_HIP(c0, launch_set_u32(b->d_frame, frame, b->stream));
    RLC_HIP(c0, hipGraphLaunch(b->exec, b->stream));
    b->next_frame = frame + 1;
    b->frame_known = true;
    return RLC_OK;
}

int rlc_batch_autotune(rlc_batch* b, uint32_t passes, rlc_schedule* h_best, rlc_schedule* h_cands, double* h_ms,
                       uint32_t* h_ncand) {
    if (!b || passes == 0) return RLC_EINVAL;
    rlc_ctx* c0 = b->scenes[0].ctx;
    std::vector<rlc_schedule> cands;
    for (uint32_t tile : {256u, 512u, 1024u, 2048u})
        for (uint32_t bpc : {4u, 8u, 16u})
            for (uint32_t dyn : {0u, 1u})
                for (uint32_t srt : {0u, 1u}) cands.push_back(rlc_schedule{tile, bpc, dyn, srt});
    hipEvent_t e0 = nullptr, e1 = nullptr;
    RLC_HIP(c0, hipEventCreate(&e0));
    RLC_HIP(c0, hipEventCreate(&e1));
    std::vector<double> ms(cands.size(), 0.0);
    size_t best = 0;
    int r = RLC_OK;
    for (size_t i = 0; i < cands.size() && r == RLC_OK; ++i) {
        for (auto& sc : b->scenes) r = r == RLC_OK ? reset_cells(sc.ctx) : r;
        if (r == RLC_OK) r = rlc_batch_set_schedule(b, &cands[i]);
        if (r == RLC_OK) r = rlc_batch_frame(b, 0);  // warm-up pass
        if (r != RLC_OK) break;
        hipError_t e = hipEventRecord(e0, b->stream);
        for (uint32_t f = 1; e == hipSuccess && f <= passes; ++f)
            e = rlc_batch_frame(b, f) == RLC_OK ? hipSuccess : hipErrorUnknown;
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) r = fail(c0, RLC_EHIP, "autotune timing: %s", hipGetErrorString(e));
        ms[i] = (double)t / passes;
        if (ms[i] < ms[best]) best = i;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != RLC_OK) return r;
    for (auto& sc : b->scenes) RLC_TRY(reset_cells(sc.ctx));
    RLC_TRY(rlc_batch_set_schedule(b, &cands[best]));
    b->frame_known = false;
    if (h_best) *h_best = cands[best];
    if (h_ncand) {
        uint32_t cap = *h_ncand;
        for (uint32_t i = 0; i < cands.size() && i < cap; ++i) {
            if (h_cands) h_cands[i] = cands[i];
            if (h_ms) h_ms[i] = ms[i];
        }
        *h_ncand = (uint32_t)cands.size();
    }
    return RLC_OK;
}

}  // extern "C"
