/*
 * rlc.h - C ABI of librlc, a HIP (gfx950) implementation of the per-frame
 * hot path of Reinforcement Lightcuts Learning (J. Pantaleoni, "Importance
 * Sampling of Many Lights with Reinforcement Lightcuts Learning",
 * arXiv:1911.10217).
 *
 * The calls follow the paper's statement of the method (section 3):
 *   build the reference light tree          rlc_build_light_tree
 *   place occluders for shadow rays          rlc_set_occluders
 *   sample a cluster and a light per point   rlc_sample
 *   shade: shadow ray, contribution, estimate rlc_shade
 *   learn: Eq. 1 statistics per cluster      rlc_learn
 *   adapt cuts: Eq. 1, split-collapse, Eq. 2 rlc_adapt_cuts
 *   all of the above for one frame            rlc_frame
 *
 * Conventions
 *  - Every pointer named d_* is DEVICE memory owned by the caller (e.g. a
 *    torch tensor's data_ptr()); it must stay valid until the work enqueued
 *    on the context's stream has completed.  Pointers named h_* are host
 *    memory.  The library owns every internal buffer.
 *  - All calls only enqueue work on the context's stream (a hipStream_t,
 *    passed as void*), except where a call says it synchronises.
 *  - Return value: RLC_OK (0) or a negative error code; rlc_last_error()
 *    gives a message.  Errors detected on the device (hash table full,
 *    non-finite contributions) are latched and reported by the next call
 *    that synchronises (rlc_sync, the dump calls).  No C++ exception crosses
 *    this interface.  A context must not be used from two threads at once.
 *  - Arrays of 3-vectors are packed float triples (x y z), row-major.
 */
#ifndef RLC_H
#define RLC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RLC_OK 0
#define RLC_EINVAL (-1)    /* bad argument, non-finite input, N == 0 ... */
#define RLC_ENOMEM (-2)    /* device allocation failed */
#define RLC_EHIP (-3)      /* a HIP runtime call failed */
#define RLC_ECAPACITY (-4) /* the cell hash table overflowed */
#define RLC_ESTATE (-5)    /* calls out of order (e.g. sample before build) */

#define RLC_MMAX 256u      /* largest supported cut size */
#define RLC_SPLIT_STEPS_MAX 65536u /* largest split_steps */

typedef struct rlc_ctx rlc_ctx;

/* Parameters of the method.  M, alpha and T are the paper's (section 3:
 * cut size, learning rate of Eq. 1, split-collapse threshold); the rest fix
 * the readings of points the paper leaves open. */
typedef struct rlc_config {
    uint32_t M;            /* cut size, 1..RLC_MMAX */
    float alpha;           /* Eq. 1 learning rate */
    float T;               /* split when Q(l_max) > T * Q(p_min) */
    float eps;             /* Q~ = Q + eps * sum(Q) / M before Eq. 2 */
    uint32_t fx_shift;     /* a reward r enters the sums as rint(min(r, reward_max) * 2^fx_shift) */
    float reward_max;
    float t_lo;            /* shadow rays cover t in (t_lo, 1 - t_lo) of x -> y */
    uint32_t reward_mode;  /* 0: reward |c_l|; 1: |c_l| * cluster size */
    uint32_t two_sided;    /* 1: emitters radiate from both faces */
    float albedo;          /* Lambertian receivers, f_r = albedo / pi */
    float grid_lo[3];      /* cell grid box; points outside clamp to the border */
    float grid_hi[3];
    uint32_t grid_dims[3];
    uint32_t hashed;       /* 0: dense grid table; 1: open-addressing hash */
    uint32_t capacity;     /* hashed: lookup slots (rounded up to 2^k, at least 64) */
    uint32_t adapt;        /* 1: split-collapse at the end of every pass */
    uint32_t temporal;     /* 0: every pass restarts from the initial cut */
    uint32_t scene_id;     /* upper key bits and RNG stream of this scene */
    uint32_t occ_grid_res; /* 0: test every box per shadow ray; n: n^3 grid, n <= 256 */
    uint32_t split_steps;  /* split-collapse steps per pass (section 3): 0 or 1, one
                              step (the basic algorithm); n > 1, repeated until a
                              step changes nothing, at most n times (with T >= 1
                              the repetition reaches that point: sum(Q^2) falls
                              at every step), 1..RLC_SPLIT_STEPS_MAX */
    uint64_t seed;         /* Philox4x32-10 key */
    uint32_t normal_bits;  /* section 3's 5-D cells: the normal's octahedral map (Cigolle et
                              al. 2014) cut into 2^normal_bits bins per coordinate, 0..8
                              (0: cells over position only).  Cell count, positions times
                              normal bins, must fit 32 bits (and 2^28 for a dense table) */
    float jitter;          /* 0..1: each sample looks up its cell from its position moved
                              by up to jitter/2 cells in the tangent plane (basis of Duff
                              et al. 2017) and its normal coordinates moved by up to
                              jitter/2 bins, drawn from Philox tag 4; 0: no jitter */
    uint32_t footprint_levels; /* section 3's footprint-sized position cells: with per-point
                              footprints set (rlc_set_footprints), levels 0..n-1 of cells
                              2^level finest cells wide, 0..16 (0 and 1: the fixed grid).
                              The cell count over all levels must fit 32 bits */
    float footprint_tile;  /* a point's level is the smallest whose cell edge (the grid's
                              smallest cell edge times 2^level) reaches footprint_tile
                              times its footprint (the coarsest if none does); > 0 when
                              footprint_levels > 1 */
    uint32_t max_cells;    /* cells the tables hold rows for (section 3's bounded memory per
                              cell: the per-cluster tables take max_cells * M * 32 bytes);
                              0: one row per lookup slot (hashed) or per cell of the grid
                              (dense); at most that many.  From 4,096 rows on, the pool is
                              cut into stripes of about 1,024 rows (up to 64), a cell taking
                              its row from the stripe its lookup slot selects.  A cell whose
                              stripe is full is not learned from, and the pass reports
                              RLC_ECAPACITY */
} rlc_config;

/* Per-sample records of rlc_sample (device arrays of n = P * spp entries,
 * sample i = point * spp + k).  Any member may be NULL where the later steps
 * do not need it (cell, slot, light and inv_pdf feed rlc_shade/rlc_learn). */
typedef struct rlc_samples {
    uint64_t* d_key;       /* cell key: (scene_id << 32) | linear cell index */
    uint32_t* d_cell;      /* internal table row of the cell (0xFFFFFFFF: none) */
    uint32_t* d_ready;     /* 1 if the cell's learned table was used */
    uint32_t* d_slot;      /* cluster s drawn from the cell's cdf */
    uint32_t* d_light;     /* light index in tree order */
    float* d_inv_pdf;      /* 1 / p(light) */
    float* d_y;            /* point on the light, 3 floats per sample */
    uint32_t* d_comp;      /* 1 if the learned proposal drew the light (mixture on);
                              rlc_learn skips those samples */
} rlc_samples;

/* Create a context whose work goes to `stream` (hipStream_t).  Allocates
 * the cell tables: 8 bytes per lookup slot (hashed: capacity; dense: every
 * cell of the grid) and M * 32 + 8 bytes per row (max_cells rows).  Rows are
 * handed out in creation order, so the rows in use are packed from row 0. */
int rlc_create(const rlc_config* cfg, void* stream, rlc_ctx** out);
int rlc_destroy(rlc_ctx* ctx);

/* Section 3 / 3.1: sort the N emissive triangles (d_tri: N x 9 floats,
 * v0 v1 v2; d_emit: N x 3 RGB) by the Morton code of their vertex sums and
 * build the binary radix tree over them, then the breadth-first initial cut
 * of min(M, N) nodes.  Resets every cell.  Synchronises (validates input). */
int rlc_build_light_tree(rlc_ctx* ctx, const float* d_tri, const float* d_emit, uint32_t N);
/* The tree's light order (section 3.1): d_perm[j] (device, N entries) is
 * the input index of the light at position j, the order of the leaves and
 * of every node's light range.  Enqueued on the context's stream. */
int rlc_get_light_order(rlc_ctx* ctx, uint32_t* d_perm);

/* Forget every cell (keys, cuts, Q, statistics): the next pass starts from
 * the initial cut everywhere, as after rlc_build_light_tree. */
int rlc_reset_cells(rlc_ctx* ctx);

/* Replace the emission of every light (d_emit: N x 3, input order); the tree
 * and the cuts are kept.  Used for animated lights. */
int rlc_set_emission(rlc_ctx* ctx, const float* d_emit, uint32_t N);

/* Occluders for the shadow rays: K axis-aligned boxes (d_aabb: K x 6, min
 * xyz then max xyz).  With occ_grid_res > 0 a uniform grid over the boxes is
 * built on the device.  Synchronises (validates input). */
int rlc_set_occluders(rlc_ctx* ctx, const float* d_aabb, uint32_t K);

/* Section 3: for every sample, locate (or create) the cell of the point,
 * draw a cluster from the cell's cdf C by binary search (cells created in
 * this pass use the initial cut, all clusters equally likely), a light
 * uniformly inside it, and a uniform point on that light.  d_nrm (P x 3) is
 * read only for 5-D cells or jitter (normal_bits > 0 or jitter > 0), and
 * may be NULL otherwise. */
int rlc_sample(rlc_ctx* ctx, const float* d_pos, const float* d_nrm, uint32_t P, uint32_t spp,
               uint32_t frame, const rlc_samples* out);

/* Shadow ray, contribution c_l = Le f_r G A V and estimate c_l / p(l) for
 * every sample.  d_radiance (P x 3) receives the mean estimate per point;
 * d_contrib (n x 3, may be NULL) c_l; d_reward (n, may be NULL) the scalar
 * reward |c_l| (times the cluster size in reward_mode 1). */
int rlc_shade(rlc_ctx* ctx, const float* d_pos, const float* d_nrm, uint32_t P, uint32_t spp,
              const rlc_samples* in, float* d_radiance, float* d_contrib, float* d_reward);

/* Eq. 1 statistics: add every sample's fixed-point reward and a count to its
 * (cell, cluster) in integer arithmetic (order-independent). */
int rlc_learn(rlc_ctx* ctx, const rlc_samples* in, const float* d_reward, uint32_t n);

/* End of a rendering pass (section 3): for every cell that received samples,
 * Q <- (1-alpha)^n Q + (1 - (1-alpha)^n) mean(r) per cluster (Eq. 1 over the
 * pass), split-collapse (one step, or up to split_steps of them), Q~ and the
 * cdf C by Eq. 2; clears the statistics. */
int rlc_adapt_cuts(rlc_ctx* ctx);

/* One whole pass: sample, shade and learn fused in one kernel, then
 * rlc_adapt_cuts.  d_radiance: P x 3. */
int rlc_frame(rlc_ctx* ctx, const float* d_pos, const float* d_nrm, uint32_t P, uint32_t spp,
              uint32_t frame, float* d_radiance);

/* One frame rendered as n_sub passes, the cuts adapted after each (section
 * 3: a frame split into sub-frames is rendered pass by pass).  Pass j =
 * 0..n_sub-1 is rlc_frame with spp / n_sub samples per point and pass index
 * frame * n_sub + j; d_radiance (P x 3) receives the passes' radiance summed
 * in pass order, times 1 / n_sub.  spp must be a multiple of n_sub, and
 * frame * n_sub + n_sub - 1 must fit in 32 bits (RLC_EINVAL otherwise).
 * n_sub = 1 is rlc_frame.  The passes' own radiance goes through a P x 3
 * buffer the context allocates on first use (and grows when P does). */
int rlc_frame_sub(rlc_ctx* ctx, const float* d_pos, const float* d_nrm, uint32_t P, uint32_t spp,
                  uint32_t n_sub, uint32_t frame, float* d_radiance);

/* Footprint-sized cells (section 3: position cells sized from the ray
 * footprint given by the area pdf of the shading point, about a tile for
 * visible points) for the following passes: d_fp[p] (`rows` floats, finite,
 * >= 0, device) is the side of point p's footprint, e.g. for a primary hit
 * the square root of the surface area its pixel covers.  The point's level
 * L is the smallest below footprint_levels whose cell edge reaches
 * footprint_tile * d_fp[p]; at level L each axis holds cells of 2^L finest
 * cells (index: the finest index shifted right by L), the jittered lookup
 * moves by up to jitter/2 of those cells, and the cell key is the
 * level-major linear index: the cells of all finer levels first, then
 * ix + dx_L (iy + dy_L (iz + dz_L (qu + 2^b qv))), dx_L = ((dx - 1) >> L) + 1.
 * Passes over more than `rows` points are refused.  d_fp = NULL: every
 * point at the finest level.  Checks the values (synchronises); the array
 * must stay valid while set. */
int rlc_set_footprints(rlc_ctx* ctx, const float* d_fp, uint32_t rows);

/* rlc_frame_sub for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same passes and results, with the passes' own radiance
 * in a fixed array of the library (32 MiB per GPU, held from the first
 * context created on that GPU until the process ends) instead of a buffer
 * the context allocates.  P at most RLC_NOALLOC_MAX_POINTS (RLC_EINVAL
 * beyond).  It allocates nothing and records no timing events.  Every call
 * on one GPU shares that array: calls that overlap on one GPU (several
 * streams, or contexts on several threads) race and must be ordered by the
 * caller. */
#define RLC_NOALLOC_MAX_POINTS 2796202u
int rlc_frame_sub_noalloc(rlc_ctx* ctx, const float* d_pos, const float* d_nrm, uint32_t P, uint32_t spp,
                          uint32_t n_sub, uint32_t frame, float* d_radiance);

/* Shadow-ray test only: d_vis[i] = 1 if the segment d_x[i] -> d_y[i] is
 * unoccluded over t in (t_lo, 1 - t_lo). */
int rlc_visible(rlc_ctx* ctx, const float* d_x, const float* d_y, uint32_t n, uint8_t* d_vis);

/* Keys of the points' position cells, (scene_id << 32) | ix + dx (iy + dy iz):
 * no normal bins, no jitter (d_keys: n entries, device). */
int rlc_cell_keys(rlc_ctx* ctx, const float* d_pos, uint32_t n, uint64_t* d_keys);

/* Error statistics of an image against a reference, FP64 on the device:
 * h_out[0..4] = mean(img), variance(img), MSE, mean relative squared error
 * (over entries with ref != 0), max abs error; n = number of floats. */
int rlc_image_error(rlc_ctx* ctx, const float* d_img, const float* d_ref, uint32_t n, double* h_out);

/* ---- batched passes over several scenes ----
 * One persistent kernel renders a pass of every scene of the batch (work
 * items of `tile` samples drawn across all scenes), then one kernel adapts
 * every scene's cells; both are captured once in a hipGraph and replayed
 * each pass.  Results are identical to rlc_frame on each scene.  All scenes'
 * contexts must use the batch's stream; the pointers are fixed at creation
 * (static points); emission may still change between passes.  Rebuild the
 * batch after rebuilding a scene's tree or occluders. */
typedef struct rlc_batch rlc_batch;

typedef struct rlc_batch_scene {
    rlc_ctx* ctx;          /* scene with its tree (and occluders) set */
    const float* d_pos;    /* P x 3 */
    const float* d_nrm;    /* P x 3 */
    float* d_radiance;     /* P x 3, the pass's mean estimate per point */
    uint32_t P;
    uint32_t spp;          /* a power of two, at most 64 */
} rlc_batch_scene;

typedef struct rlc_schedule {
    uint32_t tile;          /* samples per work item, a multiple of 256 */
    uint32_t blocks_per_cu; /* persistent blocks launched per compute unit */
    uint32_t dynamic;       /* 1: blocks take items from a counter; 0: contiguous ranges */
    uint32_t cell_sorted;   /* 1: points visited in cell order (wave-per-cell locality) */
} rlc_schedule;

int rlc_batch_create(const rlc_batch_scene* scenes, uint32_t n, void* stream, rlc_batch** out);
int rlc_batch_destroy(rlc_batch* b);
int rlc_batch_set_schedule(rlc_batch* b, const rlc_schedule* sched);
int rlc_batch_get_schedule(rlc_batch* b, rlc_schedule* sched);
/* Time every candidate schedule over `passes` passes (HIP events), keep the
 * fastest, then reset every scene's cells.  h_ms (may be NULL) receives the
 * mean pass time of each candidate, in the order of h_cands (may be NULL);
 * both hold up to *h_ncand entries on entry and the count on return. */
int rlc_batch_autotune(rlc_batch* b, uint32_t passes, rlc_schedule* h_best, rlc_schedule* h_cands, double* h_ms,
                       uint32_t* h_ncand);
/* One pass of every scene (graph launch). */
int rlc_batch_frame(rlc_batch* b, uint32_t frame);

/* ---- learned proposal (an extension beyond the paper's method) ----
 * A small network maps a point's position and normal to a distribution over
 * the nodes of a fixed breadth-first cut of up to 64 nodes of the light tree
 * (the first min(64, N) nodes that the initial-cut rule of section 3 gives
 * for M = 64).  Inputs: the position normalised to the cell-grid box and
 * the normal, each coordinate v encoded as sin / cos of 2^k pi v for
 * k = 0..11 (144 values, value 24 c + 2 k + {0: sin, 1: cos}); three hidden
 * layers of 64 ReLU units; 64 logits; softmax.  Parameters, FP32, flat:
 * W1 [64][144], b1 [64], W2 [64][64], b2, W3 [64][64], b3, W4 [64][64], b4
 * (row = output unit): RLC_MLP_PARAMS floats.  The network computes with
 * BF16 weights, inputs and activations and FP32 sums (matrix cores).
 *
 * Sampling with the mixture on (rlc_set_mixture): each sample draws from the
 * network's distribution with probability w (the network's share; a node,
 * then a light in it uniformly) and from the cell's cut otherwise, choosing
 * by Philox at counter (point, sample, frame, scene_id << 16 | 1): the
 * network when its first word, as a unit float, is below w.  Its density is
 * p(l) = (1 - w) p_cut(l) + w q(node(l)) / size(node(l)), positive for every
 * light since w < 1 and the cut's Q~ > 0, so the estimate stays unbiased for
 * any network.  Only draws from the cut feed Eq. 1.
 *
 * Training: minibatch Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the
 * weighted cross-entropy -sum_i w_i log q(x_i)[node_i] / sum_i w_i over
 * logged tuples (point, fixed-cut node, w = (c_l summed over RGB) / p(l)).
 * Epoch e visits the tuples in the order rlc_mlp_order gives (a keyed
 * permutation computed per position), in batches of `batch`; each batch is
 * one Adam step. */
#define RLC_MLP_PARAMS 21760u
#define RLC_MLP_NODES 64u

/* The fixed cut (node ids, cluster ends in tree order; up to 64). Synchronises. */
int rlc_mlp_fixed_cut(rlc_ctx* ctx, uint32_t* h_node, uint32_t* h_end, uint32_t* h_m);
/* Weights uniform in +-sqrt(6 / fan_in) from Philox at counter
 * (parameter index, 0, 0, scene_id << 16 | 3) under key `seed`; biases 0.
 * Resets Adam. */
int rlc_mlp_init(rlc_ctx* ctx, uint64_t seed);
/* Copy RLC_MLP_PARAMS floats in (resets Adam; synchronises, rejects
 * non-finite values) or out. */
int rlc_mlp_set_params(rlc_ctx* ctx, const float* d_params);
int rlc_mlp_get_params(rlc_ctx* ctx, float* d_params);
/* dst takes src's network weights, without synchronising: on dst's stream,
 * after all work enqueued so far on src's stream (an event joins the two
 * streams when they differ), so a network trained on one context's stream
 * can serve another's passes while those go on.  Resets dst's Adam state.
 * RLC_ESTATE if src has no weights. */
int rlc_mlp_copy_params(rlc_ctx* dst, rlc_ctx* src);
/* Forward pass for P points: d_cdf (P x 64, may be NULL) the inclusive
 * running sums of the 64 probabilities, left to right in FP32 (the table
 * the mixture draws from); d_logits (P x 64, may be NULL). */
int rlc_mlp_forward(rlc_ctx* ctx, const float* d_pos, const float* d_nrm, uint32_t P, float* d_cdf,
                    float* d_logits);
/* Gradient of the loss over the n tuples (d_pid[i] < P indexes d_pos/d_nrm,
 * d_node[i] < 64, d_w[i] >= 0) into d_grad (RLC_MLP_PARAMS floats); the
 * weights are unchanged.  h_loss (may be NULL) receives the loss.
 * Synchronises; bad tuples give RLC_EINVAL. */
int rlc_mlp_grad(rlc_ctx* ctx, const float* d_pos, const float* d_nrm, uint32_t P, const uint32_t* d_pid,
                 const uint32_t* d_node, const float* d_w, uint32_t n, float* d_grad, float* h_loss);
/* The order in which epoch `epoch` of rlc_mlp_train visits n tuples (the
 * paper does not fix one): d_order[i] (device, n entries) is the tuple at
 * position i, a permutation of 0..n-1 keyed by the context's seed, scene
 * id and the epoch (an eight-round Feistel network with cycle walking over
 * Philox round keys).  Enqueued on the context's stream. */
int rlc_mlp_order(rlc_ctx* ctx, uint32_t n, uint32_t epoch, uint32_t* d_order);
/* `epochs` epochs of minibatch Adam at learning rate lr over the n tuples.
 * With h_loss non-NULL the call synchronises, reports bad tuples and
 * returns the last batch's loss; with h_loss NULL it only enqueues, and bad
 * tuples are reported by the next synchronising call. */
int rlc_mlp_train(rlc_ctx* ctx, const float* d_pos, const float* d_nrm, uint32_t P, const uint32_t* d_pid,
                  const uint32_t* d_node, const float* d_w, uint32_t n, uint32_t epochs, uint32_t batch,
                  float lr, float* h_loss);
/* Mixture for the following rlc_frame / rlc_sample calls: d_cdf holds
 * `rows` rows of 64 running sums (row = point index of the pass; e.g. from
 * rlc_mlp_forward), non-decreasing with a positive last used entry; w in
 * [0, 1) is the network's share (0.5: the 50/50 mixture).  w = 0 or
 * d_cdf = NULL turns the mixture off: the plain tabular method, bit for
 * bit.  w >= 1 is RLC_EINVAL (the network alone may give a light density
 * 0).  The array must stay valid while the mixture is on.  Batched passes
 * ignore it. */
int rlc_set_mixture(rlc_ctx* ctx, const float* d_cdf, uint32_t rows, float w);
/* Training records of the following rlc_frame calls: for sample k of point
 * p, entry p * spp + k receives the point index, the fixed-cut node of the
 * drawn light and w = (c_l summed over RGB) / p(l).  `capacity` entries;
 * all NULL turns logging off.  Batched passes ignore it. */
int rlc_set_sample_log(rlc_ctx* ctx, uint32_t* d_pid, uint32_t* d_node, float* d_w, uint64_t capacity);

/* ---- inspection, checkpoint and parity interface (synchronise) ---- */
int rlc_sync(rlc_ctx* ctx);
const char* rlc_last_error(const rlc_ctx* ctx);
/* Cells created (at most the config's max_cells rows). */
int rlc_num_cells(rlc_ctx* ctx, uint32_t* h_n);
int rlc_meff(rlc_ctx* ctx, uint32_t* h_meff);
/* All cells in increasing key order; per-cell arrays have Meff columns;
 * any pointer may be NULL; `max_cells` bounds the rows written. */
int rlc_dump_cells(rlc_ctx* ctx, uint32_t max_cells, uint64_t* h_keys, uint32_t* h_ready,
                   uint32_t* h_node, uint32_t* h_end, float* h_Q, float* h_Qt, float* h_C,
                   uint64_t* h_sum, uint32_t* h_cnt);
/* Checkpoint and resume (section 3: a cell's cut and Q persist from pass
 * to pass): load n cells' learned state, as rlc_dump_cells gives it for
 * ready cells.  Host arrays: h_keys[n], keys of this context's scene, each
 * once; h_node[n x Meff], each row a cut whose nodes, in range order,
 * partition the lights (the first starts at light 0, each next one right
 * after the previous one ends, the last ends at light N-1); h_Q[n x Meff],
 * finite and >= 0.  Per cell the cluster ends follow from the tree and Q~
 * and C from Eq. 2, as at the end of a pass; the statistics start at zero;
 * the cell samples from its own table from the next pass on; an existing
 * cell is overwritten.  RLC_EINVAL (nothing loaded) for a key of another
 * scene or outside the grid, a repeated key, a cut that is not a partition
 * or a bad Q; RLC_ECAPACITY if the hash table fills.  Synchronises. */
int rlc_load_cells(rlc_ctx* ctx, uint32_t n, const uint64_t* h_keys, const uint32_t* h_node, const float* h_Q);

/* Tree arrays: perm[N] (tree order -> input index), left/right[N-1],
 * parent/first/last[2N-1] (internal nodes 0..N-2, leaf j is N-1+j),
 * rec[N x 16] = v0 v1 v2 Le area normal per light in tree order. */
int rlc_dump_tree(rlc_ctx* ctx, uint32_t* h_perm, uint32_t* h_left, uint32_t* h_right,
                  uint32_t* h_parent, uint32_t* h_first, uint32_t* h_last, float* h_rec);
int rlc_get_template(rlc_ctx* ctx, uint32_t* h_node, uint32_t* h_end, uint32_t* h_meff);

/* Per-kernel timing with HIP events on the context's stream: while enabled,
 * rlc_frame records the fused kernel and the adapt kernel separately.
 * rlc_get_timing synchronises and returns the summed milliseconds and the
 * number of frames since the last call. */
int rlc_set_timing(rlc_ctx* ctx, int enable);
int rlc_get_timing(rlc_ctx* ctx, double* h_ms_fused, double* h_ms_adapt, uint32_t* h_frames);
/* The same for rlc_mlp_train: summed milliseconds of the forward+backward
 * kernels and of the Adam updates, and the number of steps. */
int rlc_get_mlp_timing(rlc_ctx* ctx, double* h_ms_fwd_bwd, double* h_ms_update, uint32_t* h_steps);

#ifdef __cplusplus
}
#endif
#endif /* RLC_H */
