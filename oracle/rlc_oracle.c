/*
 * CPU oracle for Reinforcement Lightcuts Learning
 * (J. Pantaleoni, "Importance Sampling of Many Lights with Reinforcement
 * Lightcuts Learning", arXiv:1911.10217).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the product library never links
 * or calls it, and it shares no source, header or table with the GPU code.
 *
 * Two modes:
 *   mirror mode  - the method's per-frame loop written step by step in the
 *                  paper's order (section 3), in FP32 with an explicit
 *                  operation order (built with -ffp-contract=off, no fast
 *                  math), so that tree, cuts, Q, Q~ and C can be compared
 *                  bit for bit with any other implementation of the same
 *                  definition.
 *   truth mode   - the quantity the method estimates, direct illumination
 *                  L(x) = sum_l int_{T_l} f_r Le_l G V dA, in FP64: a closed
 *                  form (Lambert's polygon formula) for the unoccluded case
 *                  and brute-force stratified integration with visibility.
 *
 * Single threaded on purpose.  Each function names the passage it follows.
 * Readings of points where the paper is silent are marked "reading:".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_MMAX 256u
#define ORC_NONE 0xFFFFFFFFu
#define ORC_MIX_M 64u

/* ------------------------------------------------------------------------ */
/* Configuration (mirrors the method's parameters: M, alpha, T of section 3) */
/* ------------------------------------------------------------------------ */
typedef struct orc_config {
    uint32_t M;            /* cut size: every cell's cut has M nodes (section 3) */
    float alpha;           /* learning rate of Eq. 1 */
    float T;               /* split-collapse threshold (section 3) */
    float eps;             /* reading: defensive floor mixed into Q before Eq. 2 */
    uint32_t fx_shift;     /* fixed-point fraction bits of one reward */
    float reward_max;      /* rewards are clamped to this before quantisation */
    float t_lo;            /* shadow segment is t in (t_lo, 1 - t_lo) */
    uint32_t reward_mode;  /* 0: |c_l| literally; 1: |c_l| * cluster size */
    uint32_t two_sided;    /* emitters radiate from both faces */
    float albedo;          /* Lambertian receiver, f_r = albedo / pi */
    float grid_lo[3];
    float grid_hi[3];
    uint32_t grid_dims[3];
    uint32_t adapt;        /* run split-collapse at the end of each pass */
    uint32_t temporal;     /* 0: every pass restarts from the initial cut */
    uint32_t scene_id;     /* high bits of cell keys and of the RNG tag */
    uint32_t split_steps;  /* split-collapse steps per pass: 0 or 1 one step; n > 1
                              repeated until a step changes nothing, at most n */
    uint64_t seed;         /* Philox key */
    uint32_t normal_bits;  /* 5-D cells: 2^b bins per octahedral normal coordinate (0: position only) */
    float jitter;          /* jitter of the cell lookup, in cells and normal bins (0: none) */
    uint32_t footprint_levels; /* footprint-sized cells: levels 0..n-1 of cell edge base 2^level (0, 1: off) */
    float footprint_tile;  /* a point's cell edge is wanted at least tile x its footprint */
} orc_config;

#define ORC_MAX_LEVELS 16u

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator, from its published definition     */
/* (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,  */
/* 3", SC'11): ten rounds of two 32x32->64 multiplies with a fixed word     */
/* permutation, the key bumped by the Weyl constants between rounds.        */
/* ------------------------------------------------------------------------ */
static void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

int orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, uint32_t n)
{
    for (uint32_t i = 0; i < n; ++i) philox4x32_10(ctr + 4 * i, key, out + 4 * i);
    return ORC_OK;
}

/* A uniform float in [0,1) from the top 24 bits of a word. */
static float unit_float(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

/* ------------------------------------------------------------------------ */
/* Scene state                                                              */
/* ------------------------------------------------------------------------ */
typedef struct cell {
    uint32_t ready;        /* 0: created this pass, samples from the initial cut */
    uint32_t node[ORC_MMAX];
    uint32_t end[ORC_MMAX];
    float Q[ORC_MMAX];
    float Qt[ORC_MMAX];
    float C[ORC_MMAX];
    uint64_t sum[ORC_MMAX];
    uint32_t cnt[ORC_MMAX];
} cell;

typedef struct orc_ctx {
    orc_config cfg;
    uint32_t N, K;
    /* reference tree over the lights (section 3, section 3.1) */
    uint32_t* perm;        /* tree order -> input index */
    uint32_t* left;        /* internal node -> child id */
    uint32_t* right;
    uint32_t* parent;      /* any node id -> parent id (root: ORC_NONE) */
    uint32_t* first;       /* any node id -> first light (tree order) */
    uint32_t* last;        /* any node id -> last light (tree order) */
    float* rec;            /* per light in tree order: v0 v1 v2 Le A n (16 floats) */
    float* boxes;          /* K x 6: min xyz, max xyz */
    /* initial cut, copied into every new cell (section 3) */
    uint32_t Meff;
    uint32_t tmpl_node[ORC_MMAX];
    uint32_t tmpl_end[ORC_MMAX];
    float tmpl_Qt[ORC_MMAX];
    float tmpl_C[ORC_MMAX];
    /* fixed cut of the learned proposal, and the proposal's per-point cdf */
    uint32_t fix_M;
    uint32_t fix_node[ORC_MIX_M];
    uint32_t fix_end[ORC_MIX_M];
    float* mix_cdf;        /* rows of ORC_MIX_M floats, indexed by point id; NULL: off */
    uint32_t mix_rows;
    float mix_w;           /* probability of drawing from the learned proposal */
    /* grid of cells, indexed by the cell key's linear part */
    uint32_t ncell_slots;
    cell** cells;
    float inv_cell[3];
    float f_r;
    uint32_t status;       /* ORC_STATUS_* bits raised since the last orc_status */
    /* footprint-sized cells: per point id the side of its footprint, the
     * finest cell edge, and the first linear index of every level */
    float* footprint;
    uint32_t fp_rows;
    float fp_base;
    uint32_t lvl_first[ORC_MAX_LEVELS + 1];
} orc_ctx;

#define ORC_STATUS_FX_OVERFLOW 1u  /* a (cell, cluster) fixed-point reward sum wrapped 64 bits */

/* Status bits raised since the previous call, then cleared. */
uint32_t orc_status(orc_ctx* c)
{
    uint32_t s = c->status;
    c->status = 0;
    return s;
}

static int is_leaf(const orc_ctx* c, uint32_t id) { return id >= c->N - 1u; }

static uint32_t node_size(const orc_ctx* c, uint32_t id) { return c->last[id] - c->first[id] + 1u; }

/* ------------------------------------------------------------------------ */
/* Light ingest: per-triangle area and unit normal (used by the estimator)  */
/* ------------------------------------------------------------------------ */
static void triangle_frame(const float* t, float* area, float n[3])
{
    float e1x = t[3] - t[0], e1y = t[4] - t[1], e1z = t[5] - t[2];
    float e2x = t[6] - t[0], e2y = t[7] - t[1], e2z = t[8] - t[2];
    float cx = e1y * e2z - e1z * e2y;
    float cy = e1z * e2x - e1x * e2z;
    float cz = e1x * e2y - e1y * e2x;
    float len = sqrtf((cx * cx + cy * cy) + cz * cz);
    if (len == 0.0f) {
        *area = 0.0f;
        n[0] = n[1] = n[2] = 0.0f;
        return;
    }
    float inv = 1.0f / len;
    *area = 0.5f * len;
    n[0] = cx * inv;
    n[1] = cy * inv;
    n[2] = cz * inv;
}

/* ------------------------------------------------------------------------ */
/* Reference tree: "a simple LBVH builder using the 3d positions of the     */
/* lights only" (section 3.1).  Reading: each light's position is its      */
/* vertex sum, quantised to 10 bits per axis inside the bounding box and    */
/* interleaved into a 30-bit Morton code (x highest); the light's input     */
/* index is appended so that all 64-bit keys are distinct.  The tree is the */
/* binary radix tree of the sorted keys: a node over [i, j] splits after    */
/* the last key that still shares more leading bits with key i than key j  */
/* does.  Node ids: internal nodes 0..N-2 with the root at 0, a left child  */
/* that is internal takes the id of its last light, a right child that is  */
/* internal the id of its first light; leaves are N-1+position.             */
/* ------------------------------------------------------------------------ */
static uint32_t spread10(uint32_t v)
{
    uint32_t r = 0;
    for (int b = 0; b < 10; ++b) r |= ((v >> b) & 1u) << (3 * b);
    return r;
}

static int clz64(uint64_t x)
{
    if (x == 0) return 64;
    int n = 0;
    while (!(x & 0x8000000000000000ull)) {
        x <<= 1;
        ++n;
    }
    return n;
}

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static void build_node(orc_ctx* c, const uint64_t* keys, uint32_t f, uint32_t l, uint32_t id)
{
    c->first[id] = f;
    c->last[id] = l;
    int delta = clz64(keys[f] ^ keys[l]);
    uint32_t gamma = f;
    for (uint32_t k = f; k < l; ++k)
        if (clz64(keys[f] ^ keys[k]) > delta) gamma = k;
    uint32_t N = c->N;
    uint32_t lid = (gamma == f) ? (N - 1u + f) : gamma;
    uint32_t rid = (gamma + 1u == l) ? (N - 1u + l) : (gamma + 1u);
    c->left[id] = lid;
    c->right[id] = rid;
    c->parent[lid] = id;
    c->parent[rid] = id;
    if (gamma != f) build_node(c, keys, f, gamma, lid);
    if (gamma + 1u != l) build_node(c, keys, gamma + 1u, l, rid);
}

static int build_tree(orc_ctx* c, const float* tri, const float* emit)
{
    uint32_t N = c->N;
    float lo[3], hi[3];
    float* s = (float*)malloc(sizeof(float) * 3u * N);
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * N);
    if (!s || !keys) {
        free(s);
        free(keys);
        return ORC_ENOMEM;
    }
    for (uint32_t i = 0; i < N; ++i)
        for (int a = 0; a < 3; ++a) {
            float v = (tri[9 * i + a] + tri[9 * i + 3 + a]) + tri[9 * i + 6 + a];
            s[3 * i + a] = v;
            if (i == 0 || v < lo[a]) lo[a] = v;
            if (i == 0 || v > hi[a]) hi[a] = v;
        }
    float scale[3];
    for (int a = 0; a < 3; ++a) scale[a] = (hi[a] == lo[a]) ? 0.0f : 1024.0f / (hi[a] - lo[a]);
    for (uint32_t i = 0; i < N; ++i) {
        uint32_t q[3];
        for (int a = 0; a < 3; ++a) {
            float v = floorf((s[3 * i + a] - lo[a]) * scale[a]);
            if (v > 1023.0f) v = 1023.0f;
            q[a] = (uint32_t)v;
        }
        uint32_t morton = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
        keys[i] = ((uint64_t)morton << 32) | (uint64_t)i;
    }
    qsort(keys, N, sizeof(uint64_t), cmp_u64);
    for (uint32_t j = 0; j < N; ++j) c->perm[j] = (uint32_t)(keys[j] & 0xFFFFFFFFull);
    for (uint32_t j = 0; j < 2u * N - 1u; ++j) c->parent[j] = ORC_NONE;
    for (uint32_t j = 0; j < N; ++j) {
        c->first[N - 1u + j] = j;
        c->last[N - 1u + j] = j;
    }
    if (N > 1) build_node(c, keys, 0, N - 1u, 0);
    /* emitter records in tree order */
    for (uint32_t j = 0; j < N; ++j) {
        const float* t = tri + 9u * c->perm[j];
        float* r = c->rec + 16u * j;
        for (int k = 0; k < 9; ++k) r[k] = t[k];
        for (int k = 0; k < 3; ++k) r[9 + k] = emit[3u * c->perm[j] + k];
        triangle_frame(t, &r[12], &r[13]);
    }
    free(s);
    free(keys);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Initial cut: "descending the tree in breadth first order until the       */
/* desired amount of nodes M is collected" (section 3).  Reading: the cut   */
/* is a FIFO list; each step removes the earliest-enqueued node that is not */
/* a tree leaf and appends its left then right child, until M nodes are in  */
/* the list or all are leaves.  Slots are then ordered by first light, so   */
/* the cut is "a monotonically increasing list of indices marking the end  */
/* of each cluster" (section 3).                                            */
/* ------------------------------------------------------------------------ */
/* Breadth-first cut of at most M nodes: starting from the root, the       */
/* leftmost internal node of the list is replaced by its two children until */
/* M nodes are live or only leaves remain; the result in left-to-right      */
/* (first light) order.  Returns the number of nodes.                       */
static uint32_t breadth_first_cut(const orc_ctx* c, uint32_t Mreq, uint32_t* node, uint32_t* end)
{
    uint32_t M = Mreq < c->N ? Mreq : c->N;
    uint32_t list[2 * ORC_MMAX];
    int removed[2 * ORC_MMAX];
    uint32_t len = 0, live = 0;
    list[len] = 0;  /* the root (node 0; with one light the root is leaf 0 = id 0) */
    removed[len++] = 0;
    live = 1;
    while (live < M) {
        uint32_t i = 0;
        while (i < len && (removed[i] || is_leaf(c, list[i]))) ++i;
        if (i == len) break;
        removed[i] = 1;
        list[len] = c->left[list[i]];
        removed[len++] = 0;
        list[len] = c->right[list[i]];
        removed[len++] = 0;
        live += 1;
    }
    uint32_t n = 0;
    for (uint32_t i = 0; i < len; ++i)
        if (!removed[i]) node[n++] = list[i];
    /* insertion sort by first light */
    for (uint32_t i = 1; i < n; ++i) {
        uint32_t v = node[i];
        uint32_t j = i;
        while (j > 0 && c->first[node[j - 1]] > c->first[v]) {
            node[j] = node[j - 1];
            --j;
        }
        node[j] = v;
    }
    for (uint32_t s = 0; s < n; ++s) end[s] = c->last[node[s]] + 1u;
    return n;
}

/* The initial cut every new cell starts from (section 3). */
static void initial_cut(orc_ctx* c)
{
    uint32_t n = breadth_first_cut(c, c->cfg.M, c->tmpl_node, c->tmpl_end);
    c->Meff = n;
    /* a fresh cell has Q = 0 everywhere, so its Q~ and C follow from the
     * end-of-pass rule with S = 0: every cluster equally likely. */
    for (uint32_t s = 0; s < n; ++s) {
        c->tmpl_Qt[s] = 1.0f;
        c->tmpl_C[s] = (s == 0) ? 1.0f : c->tmpl_C[s - 1] + 1.0f;
    }
    /* the fixed cut the learned proposal distributes over */
    c->fix_M = breadth_first_cut(c, ORC_MIX_M, c->fix_node, c->fix_end);
}

/* ------------------------------------------------------------------------ */
/* Context                                                                  */
/* ------------------------------------------------------------------------ */
void orc_destroy(orc_ctx* c);

orc_ctx* orc_create(const orc_config* cfg, const float* tri, const float* emit, uint32_t N,
                    const float* boxes, uint32_t K)
{
    if (!cfg || !tri || !emit || N == 0 || cfg->M == 0 || cfg->M > ORC_MMAX) return NULL;
    /* one clamped reward in fixed point fits 63 bits */
    if (!(cfg->reward_max > 0.0f) || ldexp((double)cfg->reward_max, (int)cfg->fx_shift) > 9223372036854775808.0)
        return NULL;
    /* one cell pointer per 5-D cell: at most 2^27 of them */
    if (cfg->normal_bits > 8u || !(cfg->jitter >= 0.0f && cfg->jitter <= 1.0f)) return NULL;
    if (cfg->footprint_levels > ORC_MAX_LEVELS) return NULL;
    if (cfg->footprint_levels > 1u && !(cfg->footprint_tile > 0.0f && cfg->footprint_tile <= 3.402823466e38f))
        return NULL;
    /* cells of all levels (level-major linear index) */
    uint64_t first[ORC_MAX_LEVELS + 1];
    const uint32_t nlev = cfg->footprint_levels > 1u ? cfg->footprint_levels : 1u;
    first[0] = 0;
    for (uint32_t L = 0; L < nlev; ++L) {
        uint64_t n = 1;
        for (int a = 0; a < 3; ++a) n *= (uint64_t)(((cfg->grid_dims[a] - 1u) >> L) + 1u);
        first[L + 1] = first[L] + (n << (2u * cfg->normal_bits));
    }
    if (first[nlev] > (1ull << 27)) return NULL;
    orc_ctx* c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
    if (!c) return NULL;
    c->cfg = *cfg;
    c->N = N;
    c->K = K;
    uint32_t nn = 2u * N - 1u;
    c->perm = (uint32_t*)calloc(N, sizeof(uint32_t));
    c->left = (uint32_t*)calloc(N, sizeof(uint32_t));
    c->right = (uint32_t*)calloc(N, sizeof(uint32_t));
    c->parent = (uint32_t*)calloc(nn, sizeof(uint32_t));
    c->first = (uint32_t*)calloc(nn, sizeof(uint32_t));
    c->last = (uint32_t*)calloc(nn, sizeof(uint32_t));
    c->rec = (float*)calloc(16u * N, sizeof(float));
    c->boxes = (float*)calloc(6u * (K ? K : 1u), sizeof(float));
    c->ncell_slots = (uint32_t)first[nlev];
    for (uint32_t L = 0; L <= nlev; ++L) c->lvl_first[L] = (uint32_t)first[L];
    c->cells = (cell**)calloc(c->ncell_slots ? c->ncell_slots : 1u, sizeof(cell*));
    if (!c->perm || !c->left || !c->right || !c->parent || !c->first || !c->last || !c->rec ||
        !c->boxes || !c->cells) {
        orc_destroy(c);
        return NULL;
    }
    if (K) memcpy(c->boxes, boxes, sizeof(float) * 6u * K);
    if (build_tree(c, tri, emit) != ORC_OK) {
        orc_destroy(c);
        return NULL;
    }
    initial_cut(c);
    for (int a = 0; a < 3; ++a)
        c->inv_cell[a] = (float)cfg->grid_dims[a] / (cfg->grid_hi[a] - cfg->grid_lo[a]);
    /* the finest cell edge: the smallest of the three */
    for (int a = 0; a < 3; ++a) {
        float e = (cfg->grid_hi[a] - cfg->grid_lo[a]) / (float)cfg->grid_dims[a];
        if (a == 0 || e < c->fp_base) c->fp_base = e;
    }
    c->f_r = (float)((double)cfg->albedo / 3.14159265358979323846);
    return c;
}

void orc_destroy(orc_ctx* c)
{
    if (!c) return;
    if (c->cells)
        for (uint32_t i = 0; i < c->ncell_slots; ++i) free(c->cells[i]);
    free(c->cells);
    free(c->perm);
    free(c->left);
    free(c->right);
    free(c->parent);
    free(c->first);
    free(c->last);
    free(c->rec);
    free(c->boxes);
    free(c->footprint);
    free(c->mix_cdf);
    free(c);
}

/* New emission for every light (input order); the tree and cuts stay. */
int orc_set_emission(orc_ctx* c, const float* emit)
{
    for (uint32_t j = 0; j < c->N; ++j)
        for (int k = 0; k < 3; ++k) c->rec[16u * j + 9 + k] = emit[3u * c->perm[j] + k];
    return ORC_OK;
}

int orc_get_tree(const orc_ctx* c, uint32_t* perm, uint32_t* left, uint32_t* right,
                 uint32_t* parent, uint32_t* first, uint32_t* last, float* rec)
{
    uint32_t N = c->N, nn = 2u * N - 1u;
    if (perm) memcpy(perm, c->perm, sizeof(uint32_t) * N);
    if (left && N > 1) memcpy(left, c->left, sizeof(uint32_t) * (N - 1u));
    if (right && N > 1) memcpy(right, c->right, sizeof(uint32_t) * (N - 1u));
    if (parent) memcpy(parent, c->parent, sizeof(uint32_t) * nn);
    if (first) memcpy(first, c->first, sizeof(uint32_t) * nn);
    if (last) memcpy(last, c->last, sizeof(uint32_t) * nn);
    if (rec) memcpy(rec, c->rec, sizeof(float) * 16u * N);
    return ORC_OK;
}

uint32_t orc_get_template(const orc_ctx* c, uint32_t* node, uint32_t* end)
{
    if (node) memcpy(node, c->tmpl_node, sizeof(uint32_t) * c->Meff);
    if (end) memcpy(end, c->tmpl_end, sizeof(uint32_t) * c->Meff);
    return c->Meff;
}

/* The fixed breadth-first cut of up to 64 nodes that the learned proposal
 * puts its distribution over. */
uint32_t orc_fixed_cut(const orc_ctx* c, uint32_t* node, uint32_t* end)
{
    if (node) memcpy(node, c->fix_node, sizeof(uint32_t) * c->fix_M);
    if (end) memcpy(end, c->fix_end, sizeof(uint32_t) * c->fix_M);
    return c->fix_M;
}

/* Mixture proposal: cdf holds, per point id, the inclusive running sums of
 * the learned probabilities of the fixed cut's nodes (rows of 64 floats, the
 * first fix_M used).  A light is drawn from the learned proposal with
 * probability w (the network's share) and from the cell's cut otherwise.
 * cdf = NULL or w = 0 switches it off: the plain tabular method.  w = 1 (the
 * network alone) is accepted here only to pin the proposal's own draws: a
 * node the network gives probability 0 is then never drawn. */
int orc_set_mixture(orc_ctx* c, const float* cdf, uint32_t rows, float w)
{
    free(c->mix_cdf);
    c->mix_cdf = NULL;
    c->mix_rows = 0;
    if (!cdf) return ORC_OK;
    if (!(w >= 0.0f && w <= 1.0f) || rows == 0) return ORC_EINVAL;
    if (w == 0.0f) return ORC_OK;
    c->mix_cdf = (float*)malloc(sizeof(float) * ORC_MIX_M * (size_t)rows);
    if (!c->mix_cdf) return ORC_ENOMEM;
    memcpy(c->mix_cdf, cdf, sizeof(float) * ORC_MIX_M * (size_t)rows);
    c->mix_rows = rows;
    c->mix_w = w;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Cell location.  Section 3 keys cells by a 5-D grid over shading points:  */
/* three position and two normal dimensions, found by quantising jittered   */
/* coordinates.  Readings: positions on a grid of fixed resolution (each    */
/* axis quantised by floor inside the grid box, outside points clamp to the */
/* border cells); the normal mapped to the unit square by the octahedral    */
/* map and cut into 2^normal_bits bins per coordinate; the jitter a uniform */
/* offset of up to jitter/2 cells in the tangent plane of the point and of  */
/* up to jitter/2 bins on each normal coordinate, drawn per sample (Philox  */
/* tag 4).  The key is the linear 5-D cell index, with the scene id in the  */
/* upper 32 bits; without normal bins and jitter it is the position cell.   */
/* ------------------------------------------------------------------------ */
static uint32_t axis_index(float p, float lo, float inv, uint32_t dims)
{
    float f = floorf((p - lo) * inv);
    if (!(f >= 0.0f)) return 0;
    if (f >= (float)dims) return dims - 1u;
    return (uint32_t)f;
}

/* Octahedral map of a unit vector onto [0,1]^2 (Cigolle, Donow, Evangelakos, */
/* Mara, McGuire, Meyer, JCGT 3(2) 2014): project onto |x|+|y|+|z| = 1, and */
/* for z < 0 fold the lower half over the square's diagonals.               */
static void octahedral(const float n[3], float* u, float* v)
{
    float s = (fabsf(n[0]) + fabsf(n[1])) + fabsf(n[2]);
    float px = n[0] / s;
    float py = n[1] / s;
    if (n[2] < 0.0f) {
        float fx = (1.0f - fabsf(py)) * (px >= 0.0f ? 1.0f : -1.0f);
        float fy = (1.0f - fabsf(px)) * (py >= 0.0f ? 1.0f : -1.0f);
        px = fx;
        py = fy;
    }
    *u = px * 0.5f + 0.5f;
    *v = py * 0.5f + 0.5f;
}

/* Two unit tangents of the normal n (Duff, Burgess, Christensen, Hery,     */
/* Kensler, Liani, Villemin, "Building an orthonormal basis, revisited",    */
/* JCGT 6(1) 2017).                                                          */
static void tangent_frame(const float n[3], float t[3], float b[3])
{
    float sign = n[2] >= 0.0f ? 1.0f : -1.0f;
    float a = -1.0f / (sign + n[2]);
    float bb = n[0] * n[1] * a;
    t[0] = 1.0f + sign * n[0] * n[0] * a;
    t[1] = sign * bb;
    t[2] = -sign * n[0];
    b[0] = bb;
    b[1] = sign + n[1] * n[1] * a;
    b[2] = -n[1];
}

/* Footprint-sized cells (section 3: position cells sized from the ray
 * footprint that the area pdf of the shading point gives, about a
 * user-defined tile for visible points).  Reading: the caller gives each
 * point the side f of its footprint (for a primary hit, the square root of
 * the surface area its pixel covers); the wanted cell edge is tile * f, and
 * the point's level is the smallest L < levels whose edge base 2^L reaches
 * it (base: the grid's smallest cell edge), the coarsest level if none
 * does.  Level L quantises each axis into cells of 2^L finest cells (the
 * finest index shifted right by L) with ((dims - 1) >> L) + 1 of them. */
static uint32_t point_level(const orc_ctx* c, uint32_t pid)
{
    if (!c->footprint || pid >= c->fp_rows) return 0u;
    const float want = c->cfg.footprint_tile * c->footprint[pid];
    float edge = c->fp_base;
    uint32_t L = 0;
    while (L + 1u < c->cfg.footprint_levels && edge < want) {
        edge = edge * 2.0f;
        ++L;
    }
    return L;
}

static uint32_t cell_linear(const orc_ctx* c, const float* x, const float* nrm, uint32_t pid, uint32_t k,
                            uint32_t frame)
{
    const orc_config* cfg = &c->cfg;
    const uint32_t* d = cfg->grid_dims;
    const uint32_t nb = 1u << cfg->normal_bits;
    const uint32_t L = point_level(c, pid);
    float p[3] = {x[0], x[1], x[2]};
    float u = 0.0f, v = 0.0f;
    if (cfg->normal_bits) octahedral(nrm, &u, &v);
    if (cfg->jitter > 0.0f) {
        uint32_t ctr[4] = {pid, k, frame, (uint32_t)(cfg->scene_id << 16) | 4u};
        uint32_t key[2] = {(uint32_t)(cfg->seed & 0xFFFFFFFFull), (uint32_t)(cfg->seed >> 32)};
        uint32_t w[4];
        philox4x32_10(ctr, key, w);
        float xi0 = unit_float(w[0]) - 0.5f, xi1 = unit_float(w[1]) - 0.5f;
        float t[3], b[3];
        tangent_frame(nrm, t, b);
        for (int a = 0; a < 3; ++a) {
            /* up to jitter/2 cells of the point's level */
            float reach = cfg->jitter * ((cfg->grid_hi[a] - cfg->grid_lo[a]) / (float)d[a]);
            reach = reach * (float)(1u << L);
            p[a] = x[a] + reach * (xi0 * t[a] + xi1 * b[a]);
        }
        if (cfg->normal_bits) {
            u = u + ((unit_float(w[2]) - 0.5f) * cfg->jitter) / (float)nb;
            v = v + ((unit_float(w[3]) - 0.5f) * cfg->jitter) / (float)nb;
        }
    }
    uint32_t ix = axis_index(p[0], cfg->grid_lo[0], c->inv_cell[0], d[0]) >> L;
    uint32_t iy = axis_index(p[1], cfg->grid_lo[1], c->inv_cell[1], d[1]) >> L;
    uint32_t iz = axis_index(p[2], cfg->grid_lo[2], c->inv_cell[2], d[2]) >> L;
    uint32_t qu = axis_index(u, 0.0f, (float)nb, nb);
    uint32_t qv = axis_index(v, 0.0f, (float)nb, nb);
    const uint32_t dx = ((d[0] - 1u) >> L) + 1u, dy = ((d[1] - 1u) >> L) + 1u, dz = ((d[2] - 1u) >> L) + 1u;
    return c->lvl_first[L] + (ix + dx * (iy + dy * (iz + dz * (qu + nb * qv))));
}

/* Footprint sides per point id (rows of one float, finite and >= 0), or
 * NULL to quantise every point at the finest level. */
int orc_set_footprints(orc_ctx* c, const float* fp, uint32_t rows)
{
    free(c->footprint);
    c->footprint = NULL;
    c->fp_rows = 0;
    if (!fp) return ORC_OK;
    for (uint32_t i = 0; i < rows; ++i)
        if (!(fp[i] >= 0.0f && fp[i] <= 3.402823466e38f)) return ORC_EINVAL;
    c->footprint = (float*)malloc(sizeof(float) * (rows ? rows : 1u));
    if (!c->footprint) return ORC_ENOMEM;
    memcpy(c->footprint, fp, sizeof(float) * rows);
    c->fp_rows = rows;
    return ORC_OK;
}

/* The level of each point id (what point_level gives). */
int orc_point_levels(const orc_ctx* c, uint32_t n, uint32_t* out)
{
    for (uint32_t i = 0; i < n; ++i) out[i] = point_level(c, i);
    return ORC_OK;
}

static uint64_t cell_key(const orc_ctx* c, uint32_t lin)
{
    return ((uint64_t)c->cfg.scene_id << 32) | (uint64_t)lin;
}

/* Keys of the points' position cells (no normal bins, no jitter). */
int orc_cell_keys(const orc_ctx* c, const float* pos, uint32_t P, uint64_t* keys)
{
    const uint32_t* d = c->cfg.grid_dims;
    for (uint32_t i = 0; i < P; ++i) {
        const float* p = pos + 3u * i;
        uint32_t ix = axis_index(p[0], c->cfg.grid_lo[0], c->inv_cell[0], d[0]);
        uint32_t iy = axis_index(p[1], c->cfg.grid_lo[1], c->inv_cell[1], d[1]);
        uint32_t iz = axis_index(p[2], c->cfg.grid_lo[2], c->inv_cell[2], d[2]);
        keys[i] = cell_key(c, ix + d[0] * (iy + d[1] * iz));
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Shadow ray: any-hit of the segment x -> y against axis-aligned boxes     */
/* (slab test), over t in (t_lo, 1 - t_lo); a strict tn < tf occludes.      */
/* Every box is tested: this is the brute-force definition of V.            */
/* ------------------------------------------------------------------------ */
static int segment_blocked(const orc_ctx* c, const float o[3], const float d[3])
{
    float invd[3];
    for (int a = 0; a < 3; ++a) invd[a] = 1.0f / d[a];
    for (uint32_t b = 0; b < c->K; ++b) {
        const float* box = c->boxes + 6u * b;
        float tn = c->cfg.t_lo;
        float tf = 1.0f - c->cfg.t_lo;
        int miss = 0;
        for (int a = 0; a < 3 && !miss; ++a) {
            if (d[a] == 0.0f) {
                if (o[a] < box[a] || o[a] > box[3 + a]) miss = 1;
                continue;
            }
            float t0 = (box[a] - o[a]) * invd[a];
            float t1 = (box[3 + a] - o[a]) * invd[a];
            float tmin = t0 < t1 ? t0 : t1;
            float tmax = t0 < t1 ? t1 : t0;
            if (tmin > tn) tn = tmin;
            if (tmax < tf) tf = tmax;
        }
        if (!miss && tn < tf) return 1;
    }
    return 0;
}

int orc_visible(const orc_ctx* c, const float* x, const float* y, uint32_t n, uint8_t* vis)
{
    for (uint32_t i = 0; i < n; ++i) {
        float d[3];
        for (int a = 0; a < 3; ++a) d[a] = y[3 * i + a] - x[3 * i + a];
        vis[i] = (uint8_t)!segment_blocked(c, x + 3 * i, d);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One light sample at one shading point (section 3): a cluster s drawn     */
/* from the cdf of the point's cell, one light of that cluster picked at    */
/* random, then the light's contribution c_l.                               */
/* ------------------------------------------------------------------------ */
typedef struct orc_records {
    uint64_t* key;      /* cell key */
    uint32_t* ready;    /* 1 if the cell's learned table was used */
    uint32_t* slot;     /* cluster s */
    uint32_t* light;    /* light l, tree order */
    float* inv_pdf;     /* 1 / p(l) */
    float* y;           /* point on the light, 3 per sample */
    float* contrib;     /* c_l, RGB, 3 per sample */
    float* reward;      /* scalar reward fed to Eq. 1 */
    uint32_t* fnode;    /* index of the fixed-cut node holding the light */
    float* weight;      /* training weight (c_l summed over RGB) / p(l) */
    uint32_t* comp;     /* 1 if the learned proposal drew the light */
} orc_records;

static cell* get_or_create_cell(orc_ctx* c, uint32_t lin)
{
    cell* ce = c->cells[lin];
    if (!ce) {
        ce = (cell*)calloc(1, sizeof(cell));
        c->cells[lin] = ce;  /* created now; learned tables exist from the end of the pass */
    }
    return ce;
}

static void one_sample(orc_ctx* c, const float* x, const float* nx, uint32_t pid, uint32_t k,
                       uint32_t frame, float est[3], orc_records* out, uint32_t ri)
{
    const orc_config* cfg = &c->cfg;
    uint32_t lin = cell_linear(c, x, nx, pid, k, frame);
    cell* ce = get_or_create_cell(c, lin);
    int use_cell = ce && ce->ready;
    const float* C = use_cell ? ce->C : c->tmpl_C;
    const float* Qt = use_cell ? ce->Qt : c->tmpl_Qt;
    const uint32_t* end = use_cell ? ce->end : c->tmpl_end;
    uint32_t Meff = c->Meff;

    /* random words for this sample: counter (point, sample, frame, tag 0 | scene) */
    uint32_t ctr[4] = {pid, k, frame, (uint32_t)(cfg->scene_id << 16)};
    uint32_t key[2] = {(uint32_t)(cfg->seed & 0xFFFFFFFFull), (uint32_t)(cfg->seed >> 32)};
    uint32_t w[4];
    philox4x32_10(ctr, key, w);
    float u0 = unit_float(w[0]);
    uint64_t draw40 = ((uint64_t)(w[0] & 0xFFu) << 32) | (uint64_t)w[1];
    float u2 = unit_float(w[2]);
    float u3 = unit_float(w[3]);

    /* component of the mixture: counter tag 1 (only with the proposal on) */
    const float* q = NULL;
    int use_mlp = 0;
    if (c->mix_cdf && pid < c->mix_rows) {
        uint32_t ctr1[4] = {pid, k, frame, (uint32_t)(cfg->scene_id << 16) | 1u};
        uint32_t w1[4];
        philox4x32_10(ctr1, key, w1);
        q = c->mix_cdf + (size_t)pid * ORC_MIX_M;
        use_mlp = unit_float(w1[0]) < c->mix_w;
    }
    uint32_t Mf = c->fix_M;
    uint32_t s, begin, size, l, kf = ORC_NONE, fbegin = 0, fsize = 0;
    if (!use_mlp) {
        /* cluster: smallest s with t < C[s] */
        float t = u0 * C[Meff - 1];
        s = Meff - 1;
        for (uint32_t i = 0; i < Meff; ++i)
            if (t < C[i]) {
                s = i;
                break;
            }
        begin = (s == 0) ? 0u : end[s - 1];
        size = end[s] - begin;
        /* light inside the cluster, uniformly (the paper leaves the choice open) */
        l = begin + (uint32_t)((draw40 * (uint64_t)size) >> 40);
    } else {
        /* node of the fixed cut from the learned cdf, then a light inside it
         * uniformly; the same random words as the tabular draw */
        float t = u0 * q[Mf - 1];
        kf = Mf - 1;
        for (uint32_t i = 0; i < Mf; ++i)
            if (t < q[i]) {
                kf = i;
                break;
            }
        fbegin = (kf == 0) ? 0u : c->fix_end[kf - 1];
        fsize = c->fix_end[kf] - fbegin;
        l = fbegin + (uint32_t)((draw40 * (uint64_t)fsize) >> 40);
        /* the cell's cluster that holds l */
        s = Meff - 1;
        for (uint32_t i = 0; i < Meff; ++i)
            if (l < end[i]) {
                s = i;
                break;
            }
        begin = (s == 0) ? 0u : end[s - 1];
        size = end[s] - begin;
    }
    if (kf == ORC_NONE && (q || (out && (out->fnode || out->weight)))) {
        kf = Mf - 1;
        for (uint32_t i = 0; i < Mf; ++i)
            if (l < c->fix_end[i]) {
                kf = i;
                break;
            }
        fbegin = (kf == 0) ? 0u : c->fix_end[kf - 1];
        fsize = c->fix_end[kf] - fbegin;
    }
    float inv_pdf;
    if (q) {
        /* p(l) = (1 - w) p_cut(l) + w p_learned(l), each uniform inside its
         * cluster / node */
        float pt = Qt[s] / ((float)size * C[Meff - 1]);
        float qk = q[kf] - (kf ? q[kf - 1] : 0.0f);
        float pm = qk / ((float)fsize * q[Mf - 1]);
        inv_pdf = 1.0f / ((1.0f - c->mix_w) * pt + c->mix_w * pm);
    } else {
        inv_pdf = ((float)size * C[Meff - 1]) / Qt[s];
    }

    /* uniform point on the triangle */
    const float* r = c->rec + 16u * l;
    float su = sqrtf(u2);
    float b0 = 1.0f - su;
    float b1 = u3 * su;
    float b2 = (1.0f - b0) - b1;
    float y[3];
    for (int a = 0; a < 3; ++a) y[a] = (b0 * r[a] + b1 * r[3 + a]) + b2 * r[6 + a];

    /* contribution c_l = Le * f_r * G * A * V */
    float cl[3] = {0.0f, 0.0f, 0.0f};
    float d[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
    float dist2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    float area = r[12];
    if (dist2 > 0.0f && area > 0.0f) {
        float dist = sqrtf(dist2);
        float cos_x = ((nx[0] * d[0] + nx[1] * d[1]) + nx[2] * d[2]) / dist;
        float dl = (r[13] * d[0] + r[14] * d[1]) + r[15] * d[2];
        float cos_l;
        if (cfg->two_sided)
            cos_l = fabsf(dl) / dist;
        else
            cos_l = (dl < 0.0f ? -dl : 0.0f) / dist;
        if (cos_x > 0.0f && cos_l > 0.0f) {
            float G = (cos_x * cos_l) / dist2;
            float kk = (c->f_r * G) * area;
            if (kk > 0.0f && (r[9] > 0.0f || r[10] > 0.0f || r[11] > 0.0f)) {
                if (!segment_blocked(c, x, d)) {
                    cl[0] = r[9] * kk;
                    cl[1] = r[10] * kk;
                    cl[2] = r[11] * kk;
                }
            }
        }
    }
    /* unbiased estimate c_l / p(l) */
    for (int a = 0; a < 3; ++a) est[a] = cl[a] * inv_pdf;

    /* reward |c_l| (L1 over RGB) and its fixed-point sample for Eq. 1 */
    float rew = (cl[0] + cl[1]) + cl[2];
    if (cfg->reward_mode == 1) rew = rew * (float)size;
    float rc = rew < cfg->reward_max ? rew : cfg->reward_max;
    uint64_t qfx = (uint64_t)rintf(rc * ldexpf(1.0f, (int)cfg->fx_shift));
    /* reading: only draws from the cell's own cut feed Eq. 1 (inside a
     * cluster they are uniform, as the update assumes) */
    if (ce && !use_mlp) {
        /* a 64-bit sum that wraps is flagged: its statistics are not valid */
        if (ce->sum[s] + qfx < ce->sum[s]) c->status |= ORC_STATUS_FX_OVERFLOW;
        ce->sum[s] += qfx;
        ce->cnt[s] += 1u;
    }
    if (out) {
        if (out->key) out->key[ri] = cell_key(c, lin);
        if (out->ready) out->ready[ri] = (uint32_t)use_cell;
        if (out->slot) out->slot[ri] = s;
        if (out->light) out->light[ri] = l;
        if (out->inv_pdf) out->inv_pdf[ri] = inv_pdf;
        if (out->y)
            for (int a = 0; a < 3; ++a) out->y[3 * ri + a] = y[a];
        if (out->contrib)
            for (int a = 0; a < 3; ++a) out->contrib[3 * ri + a] = cl[a];
        if (out->reward) out->reward[ri] = rew;
        if (out->fnode) out->fnode[ri] = kf;
        if (out->weight) out->weight[ri] = ((cl[0] + cl[1]) + cl[2]) * inv_pdf;
        if (out->comp) out->comp[ri] = (uint32_t)use_mlp;
    }
}

/* One rendering pass over the given points: sample, shade and accumulate   */
/* the learning statistics.  pid[i] is the global index of point i (it      */
/* keys the random numbers), so any subset of a frame's points can be run.  */
/* radiance: P x 3, the mean of the spp estimates of each point.            */
int orc_frame(orc_ctx* c, const float* pos, const float* nrm, const uint32_t* pid, uint32_t P,
              uint32_t spp, uint32_t frame, float* radiance, orc_records* out)
{
    if (spp == 0) return ORC_EINVAL;
    float inv_spp = 1.0f / (float)spp;
    for (uint32_t i = 0; i < P; ++i) {
        uint32_t g = pid ? pid[i] : i;
        float acc[3] = {0.0f, 0.0f, 0.0f};
        for (uint32_t k = 0; k < spp; ++k) {
            float e[3];
            one_sample(c, pos + 3u * i, nrm + 3u * i, g, k, frame, e, out, i * spp + k);
            for (int a = 0; a < 3; ++a) acc[a] = acc[a] + e[a];
        }
        if (radiance)
            for (int a = 0; a < 3; ++a) radiance[3u * i + a] = acc[a] * inv_spp;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Eq. 1 over one pass.  Reading: the n samples a cluster received in a     */
/* pass update Q in batch form, Q <- a^n Q + (1 - a^n) mean(r), a = 1-alpha, */
/* which is Eq. 1 itself for n = 1 and the average of Eq. 1 over all orders */
/* of the n samples for n > 1.  a^n is taken by binary exponentiation.      */
/* ------------------------------------------------------------------------ */
static float pow_uint(float a, uint32_t n)
{
    float res = 1.0f, b = a;
    while (n) {
        if (n & 1u) res = res * b;
        b = b * b;
        n >>= 1;
    }
    return res;
}

static float ema_update(float Q, uint64_t sum, uint32_t n, float alpha, uint32_t fx_shift)
{
    float a_n = pow_uint(1.0f - alpha, n);
    float m = ((float)sum * ldexpf(1.0f, -(int)fx_shift)) / (float)n;
    float t1 = a_n * Q;
    float t2 = (1.0f - a_n) * m;
    return t1 + t2;
}

int orc_ema(const float* Q, const uint64_t* sum, const uint32_t* cnt, uint32_t n, float alpha,
            uint32_t fx_shift, float* Qout)
{
    for (uint32_t i = 0; i < n; ++i) Qout[i] = cnt[i] ? ema_update(Q[i], sum[i], cnt[i], alpha, fx_shift) : Q[i];
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Split-collapse, one step (section 3 and Fig. 1).  l_max: the cut leaf    */
/* with the largest Q among those that can still be split (its node holds   */
/* at least two lights).  p_min: among the parents whose two children are   */
/* both in the cut, the one with the smallest Q, where a parent's Q is the  */
/* sum of its children's (reading).  If Q(l_max) > T Q(p_min), l_max is     */
/* replaced by its children (each with half its Q) and p_min's children by */
/* p_min (with their summed Q).  Ties go to the smallest slot; a pair that  */
/* contains l_max is not a candidate.  Returns 1 if the cut changed.        */
/* ------------------------------------------------------------------------ */
static int split_collapse(const orc_ctx* c, uint32_t* node, float* Q, uint32_t Meff, float T)
{
    if (Meff < 2) return 0;
    int smax = -1;
    for (uint32_t s = 0; s < Meff; ++s)
        if (node_size(c, node[s]) >= 2u && (smax < 0 || Q[s] > Q[smax])) smax = (int)s;
    int smin = -1;
    float qmin = 0.0f;
    for (uint32_t s = 0; s + 1u < Meff; ++s) {
        uint32_t p = c->parent[node[s]];
        if (p == ORC_NONE || c->left[p] != node[s] || c->right[p] != node[s + 1u]) continue;
        if ((int)s == smax || (int)s + 1 == smax) continue;
        float qp = Q[s] + Q[s + 1u];
        if (smin < 0 || qp < qmin) {
            smin = (int)s;
            qmin = qp;
        }
    }
    if (smax < 0 || smin < 0) return 0;
    if (!(Q[smax] > T * qmin)) return 0;
    uint32_t nn[ORC_MMAX];
    float nq[ORC_MMAX];
    uint32_t m = 0;
    for (uint32_t s = 0; s < Meff; ++s) {
        if ((int)s == smin) {
            nn[m] = c->parent[node[s]];
            nq[m++] = qmin;
        } else if ((int)s == smin + 1) {
            continue;
        } else if ((int)s == smax) {
            float h = 0.5f * Q[s];
            nn[m] = c->left[node[s]];
            nq[m++] = h;
            nn[m] = c->right[node[s]];
            nq[m++] = h;
        } else {
            nn[m] = node[s];
            nq[m++] = Q[s];
        }
    }
    memcpy(node, nn, sizeof(uint32_t) * Meff);
    memcpy(Q, nq, sizeof(float) * Meff);
    return 1;
}

int orc_split_collapse(const orc_ctx* c, uint32_t* node, float* Q, uint32_t Meff, float T)
{
    return split_collapse(c, node, Q, Meff, T);
}

/* ------------------------------------------------------------------------ */
/* Eq. 2: C(0) = Q(0), C(s) = C(s-1) + Q(s), taken over Q~.  Reading: Q~ =  */
/* Q + eps * sum(Q) / M keeps every cluster's probability positive; with    */
/* sum(Q) = 0 every cluster is equally likely (Q~ = 1).                      */
/* ------------------------------------------------------------------------ */
static void rebuild_cdf(const float* Q, uint32_t Meff, float eps, float* Qt, float* C)
{
    float S = 0.0f;
    for (uint32_t s = 0; s < Meff; ++s) S = S + Q[s];
    if (S == 0.0f) {
        for (uint32_t s = 0; s < Meff; ++s) Qt[s] = 1.0f;
    } else {
        float floor_term = (eps * S) / (float)Meff;
        /* reading: with eps > 0 every cluster keeps a positive probability.
         * Q decays geometrically under Eq. 1 when a cell's rewards stay 0,
         * and once S is tiny the floor underflows to 0; it is then held at
         * the smallest normal float, which tends to the S = 0 rule (all
         * clusters equally likely) as S -> 0. */
        if (eps > 0.0f && floor_term < 1.17549435e-38f) floor_term = 1.17549435e-38f;
        for (uint32_t s = 0; s < Meff; ++s) Qt[s] = Q[s] + floor_term;
    }
    C[0] = Qt[0];
    for (uint32_t s = 1; s < Meff; ++s) C[s] = C[s - 1] + Qt[s];
}

int orc_cdf(const float* Q, uint32_t Meff, float eps, float* Qt, float* C)
{
    rebuild_cdf(Q, Meff, eps, Qt, C);
    return ORC_OK;
}

/* End of a rendering pass: for every cell that received samples, Eq. 1,    */
/* then split-collapse, then Q~ and Eq. 2; statistics are cleared.  The     */
/* basic algorithm takes one split-collapse step; section 3 notes that it   */
/* could be repeated until no pair of nodes is touched, which split_steps   */
/* > 1 does, stopping after that many steps at the latest.                  */
int orc_adapt(orc_ctx* c)
{
    const orc_config* cfg = &c->cfg;
    uint32_t Meff = c->Meff;
    for (uint32_t lin = 0; lin < c->ncell_slots; ++lin) {
        cell* ce = c->cells[lin];
        if (!ce) continue;
        uint64_t total = 0;
        for (uint32_t s = 0; s < Meff; ++s) total += ce->cnt[s];
        if (total == 0) continue;
        if (!ce->ready || !cfg->temporal) {
            for (uint32_t s = 0; s < Meff; ++s) {
                ce->node[s] = c->tmpl_node[s];
                ce->Q[s] = 0.0f;
            }
        }
        if (cfg->temporal) {
            for (uint32_t s = 0; s < Meff; ++s)
                if (ce->cnt[s]) ce->Q[s] = ema_update(ce->Q[s], ce->sum[s], ce->cnt[s], cfg->alpha, cfg->fx_shift);
            if (cfg->adapt) {
                uint32_t steps = cfg->split_steps > 1u ? cfg->split_steps : 1u;
                for (uint32_t k = 0; k < steps; ++k)
                    if (!split_collapse(c, ce->node, ce->Q, Meff, cfg->T)) break;
            }
        }
        for (uint32_t s = 0; s < Meff; ++s) ce->end[s] = c->last[ce->node[s]] + 1u;
        rebuild_cdf(ce->Q, Meff, cfg->eps, ce->Qt, ce->C);
        memset(ce->sum, 0, sizeof(ce->sum));
        memset(ce->cnt, 0, sizeof(ce->cnt));
        ce->ready = 1;
    }
    return ORC_OK;
}

uint32_t orc_num_cells(const orc_ctx* c)
{
    uint32_t n = 0;
    for (uint32_t lin = 0; lin < c->ncell_slots; ++lin) n += c->cells[lin] != NULL;
    return n;
}

uint32_t orc_meff(const orc_ctx* c) { return c->Meff; }

/* Cells in key order; per-cell arrays are Meff wide.  Any pointer may be NULL. */
int orc_dump_cells(const orc_ctx* c, uint64_t* keys, uint32_t* ready, uint32_t* node,
                   uint32_t* end, float* Q, float* Qt, float* C, uint64_t* sum, uint32_t* cnt)
{
    uint32_t Meff = c->Meff, i = 0;
    for (uint32_t lin = 0; lin < c->ncell_slots; ++lin) {
        const cell* ce = c->cells[lin];
        if (!ce) continue;
        if (keys) keys[i] = cell_key(c, lin);
        if (ready) ready[i] = ce->ready;
        size_t o = (size_t)i * Meff;
        if (node) memcpy(node + o, ce->node, sizeof(uint32_t) * Meff);
        if (end) memcpy(end + o, ce->end, sizeof(uint32_t) * Meff);
        if (Q) memcpy(Q + o, ce->Q, sizeof(float) * Meff);
        if (Qt) memcpy(Qt + o, ce->Qt, sizeof(float) * Meff);
        if (C) memcpy(C + o, ce->C, sizeof(float) * Meff);
        if (sum) memcpy(sum + o, ce->sum, sizeof(uint64_t) * Meff);
        if (cnt) memcpy(cnt + o, ce->cnt, sizeof(uint32_t) * Meff);
        ++i;
    }
    return ORC_OK;
}

/* Overwrite one cell's learned state (creating it, ready) - test hook.    */
/* Load one cell's learned state (a checkpoint): its cut, which must be a
 * partition of the lights in range order (the first node starts at light
 * 0, each next one right after the previous one ends, the last ends at
 * N - 1), and its Q (finite, >= 0).  The ends follow from the tree and Q~,
 * C from Eq. 2, as at the end of a pass; the statistics start at zero and
 * the cell samples from its own table from the next pass on. */
int orc_load_cell(orc_ctx* c, uint32_t lin, const uint32_t* node, const float* Q)
{
    if (lin >= c->ncell_slots) return ORC_EINVAL;
    const uint32_t nn = 2u * c->N - 1u;
    uint32_t next = 0;
    for (uint32_t s = 0; s < c->Meff; ++s) {
        if (node[s] >= nn || c->first[node[s]] != next) return ORC_EINVAL;
        if (!(Q[s] >= 0.0f && Q[s] <= 3.402823466e38f)) return ORC_EINVAL;
        next = c->last[node[s]] + 1u;
    }
    if (next != c->N) return ORC_EINVAL;
    cell* ce = get_or_create_cell(c, lin);
    if (!ce) return ORC_ENOMEM;
    for (uint32_t s = 0; s < c->Meff; ++s) {
        ce->node[s] = node[s];
        ce->Q[s] = Q[s];
        ce->end[s] = c->last[node[s]] + 1u;
    }
    rebuild_cdf(ce->Q, c->Meff, c->cfg.eps, ce->Qt, ce->C);
    memset(ce->sum, 0, sizeof(ce->sum));
    memset(ce->cnt, 0, sizeof(ce->cnt));
    ce->ready = 1;
    return ORC_OK;
}

/* ======================================================================== */
/* Truth mode (FP64): the direct illumination the method estimates.         */
/* ======================================================================== */

/* int over the triangle of cos_x * |cos_l| / r^2 dA, by Lambert's formula   */
/* for a polygon (the form factor from a differential area to a polygon),   */
/* after clipping the triangle to the half-space above the tangent plane.   */
static double polygon_geometry(const double x[3], const double n[3], const double v[3][3], int two_sided,
                               const double nl[3])
{
    if (!two_sided) {
        /* a one-sided emitter radiates along its normal only */
        double w = nl[0] * (x[0] - v[0][0]) + nl[1] * (x[1] - v[0][1]) + nl[2] * (x[2] - v[0][2]);
        if (w <= 0.0) return 0.0;
    }
    double poly[8][3];
    int np = 0;
    for (int i = 0; i < 3; ++i) {
        const double* a = v[i];
        const double* b = v[(i + 1) % 3];
        double ha = n[0] * (a[0] - x[0]) + n[1] * (a[1] - x[1]) + n[2] * (a[2] - x[2]);
        double hb = n[0] * (b[0] - x[0]) + n[1] * (b[1] - x[1]) + n[2] * (b[2] - x[2]);
        if (ha > 0.0) {
            for (int k = 0; k < 3; ++k) poly[np][k] = a[k];
            ++np;
        }
        if ((ha > 0.0) != (hb > 0.0)) {
            double t = ha / (ha - hb);
            for (int k = 0; k < 3; ++k) poly[np][k] = a[k] + t * (b[k] - a[k]);
            ++np;
        }
    }
    if (np < 3) return 0.0;
    double acc = 0.0;
    for (int i = 0; i < np; ++i) {
        double r0[3], r1[3];
        for (int k = 0; k < 3; ++k) {
            r0[k] = poly[i][k] - x[k];
            r1[k] = poly[(i + 1) % np][k] - x[k];
        }
        double l0 = sqrt(r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2]);
        double l1 = sqrt(r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
        for (int k = 0; k < 3; ++k) {
            r0[k] /= l0;
            r1[k] /= l1;
        }
        double cr[3] = {r0[1] * r1[2] - r0[2] * r1[1], r0[2] * r1[0] - r0[0] * r1[2], r0[0] * r1[1] - r0[1] * r1[0]};
        double cl = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        if (cl == 0.0) continue;
        double dt = r0[0] * r1[0] + r0[1] * r1[1] + r0[2] * r1[2];
        double theta = atan2(cl, dt);
        acc += theta * (n[0] * cr[0] + n[1] * cr[1] + n[2] * cr[2]) / cl;
    }
    return 0.5 * fabs(acc);
}

/* Unoccluded direct illumination at each point (RGB), closed form. */
int orc_truth_unoccluded(const orc_ctx* c, const float* pos, const float* nrm, uint32_t P, double* out)
{
    double fr = (double)c->cfg.albedo / 3.14159265358979323846;
    for (uint32_t i = 0; i < P; ++i) {
        double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        double n[3] = {nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]};
        double acc[3] = {0.0, 0.0, 0.0};
        for (uint32_t l = 0; l < c->N; ++l) {
            const float* r = c->rec + 16u * l;
            if (r[12] == 0.0f) continue;
            double v[3][3];
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k) v[j][k] = r[3 * j + k];
            double nl[3] = {r[13], r[14], r[15]};
            double g = polygon_geometry(x, n, (const double(*)[3])v, (int)c->cfg.two_sided, nl);
            for (int k = 0; k < 3; ++k) acc[k] += fr * (double)r[9 + k] * g;
        }
        for (int k = 0; k < 3; ++k) out[3 * i + k] = acc[k];
    }
    return ORC_OK;
}

static int segment_blocked_f64(const orc_ctx* c, const double o[3], const double d[3])
{
    for (uint32_t b = 0; b < c->K; ++b) {
        const float* box = c->boxes + 6u * b;
        double tn = (double)c->cfg.t_lo, tf = 1.0 - (double)c->cfg.t_lo;
        int miss = 0;
        for (int a = 0; a < 3 && !miss; ++a) {
            if (d[a] == 0.0) {
                if (o[a] < box[a] || o[a] > box[3 + a]) miss = 1;
                continue;
            }
            double t0 = ((double)box[a] - o[a]) / d[a];
            double t1 = ((double)box[3 + a] - o[a]) / d[a];
            double lo = t0 < t1 ? t0 : t1, hi = t0 < t1 ? t1 : t0;
            if (lo > tn) tn = lo;
            if (hi < tf) tf = hi;
        }
        if (!miss && tn < tf) return 1;
    }
    return 0;
}

/* Direct illumination with visibility by stratified jittered integration */
/* over every light (ks x ks strata per triangle), FP64.  The jitter comes */
/* from Philox with tag 3 and counter (point, stratum, light).            */
/* out: P x 3.                                                             */
int orc_truth_mc(const orc_ctx* c, const float* pos, const float* nrm, const uint32_t* pid, uint32_t P,
                 uint32_t ks, uint32_t replica, double* out)
{
    double fr = (double)c->cfg.albedo / 3.14159265358979323846;
    uint32_t key[2] = {(uint32_t)(c->cfg.seed & 0xFFFFFFFFull), (uint32_t)(c->cfg.seed >> 32)};
    for (uint32_t i = 0; i < P; ++i) {
        double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        double n[3] = {nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]};
        double acc[3] = {0.0, 0.0, 0.0};
        uint32_t g = pid ? pid[i] : i;
        for (uint32_t l = 0; l < c->N; ++l) {
            const float* r = c->rec + 16u * l;
            double A = r[12];
            if (A == 0.0) continue;
            double sumG = 0.0;
            for (uint32_t a = 0; a < ks; ++a)
                for (uint32_t b = 0; b < ks; ++b) {
                    uint32_t ctr[4] = {g, a * ks + b, l, 3u | (replica << 8)};
                    uint32_t w[4];
                    philox4x32_10(ctr, key, w);
                    double u = ((double)a + ((double)w[0] + 0.5) / 4294967296.0) / (double)ks;
                    double v = ((double)b + ((double)w[1] + 0.5) / 4294967296.0) / (double)ks;
                    double su = sqrt(u);
                    double b0 = 1.0 - su, b1 = v * su, b2 = 1.0 - b0 - b1;
                    double y[3], d[3];
                    for (int k = 0; k < 3; ++k) {
                        y[k] = b0 * r[k] + b1 * r[3 + k] + b2 * r[6 + k];
                        d[k] = y[k] - x[k];
                    }
                    double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    if (d2 <= 0.0) continue;
                    double dist = sqrt(d2);
                    double cx = (n[0] * d[0] + n[1] * d[1] + n[2] * d[2]) / dist;
                    double dl = (r[13] * d[0] + r[14] * d[1] + r[15] * d[2]) / dist;
                    double cl = c->cfg.two_sided ? fabs(dl) : (dl < 0.0 ? -dl : 0.0);
                    if (cx <= 0.0 || cl <= 0.0) continue;
                    if (segment_blocked_f64(c, x, d)) continue;
                    sumG += cx * cl / d2;
                }
            double mean = sumG / ((double)ks * (double)ks);
            for (int k = 0; k < 3; ++k) acc[k] += fr * (double)r[9 + k] * A * mean;
        }
        for (int k = 0; k < 3; ++k) out[3 * i + k] = acc[k];
    }
    return ORC_OK;
}
