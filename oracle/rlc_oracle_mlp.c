/*
 * CPU oracle for the learned proposal: a small MLP that maps a shading
 * point's position and normal to a distribution over the nodes of a fixed
 * 64-node cut, mixed with the tabular cut distribution of section 3 so that
 * the estimator stays unbiased.
 *
 * TEST INFRASTRUCTURE ONLY (see rlc_oracle.c): used by the tests and never
 * by the product library; no code is shared with the GPU path.
 *
 * Everything here is FP64.  With bf16 = 1 the values the GPU kernels hold in
 * BF16 (encoded inputs, weights, hidden activations, output gradients and
 * back-propagated gradients) are rounded to BF16 at the same points, so the
 * GPU's FP32-accumulated results can be compared within BF16 tolerance.
 *
 * Network: x (144) -> 64 -> 64 -> 64 (ReLU each) -> 64 logits -> softmax.
 * Encoding: for each of the 6 inputs v (position normalised to the cell-grid
 * box, then the normal) and k = 0..11: sin(2^k pi v), cos(2^k pi v), stored
 * at index 24 c + 2 k (+1 for the cosine).
 * Parameters, flat: W1 [64][144], b1[64], W2 [64][64], b2, W3 [64][64], b3,
 * W4 [64][64], b4 (row = output unit).
 * Loss over a batch of (x_i, node k_i, weight w_i): -sum_i w_i log q_i[k_i]
 * / sum_i w_i, the one-sample estimate of the KL divergence from the target
 * distribution (proportional to the lights' contributions) to q.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IN 144
#define H 64
#define OUT 64
#define NPARAM (H * IN + H + 2 * (H * H + H) + OUT * H + OUT)

static const double PI = 3.14159265358979323846;

uint32_t orc_mlp_nparam(void) { return NPARAM; }

/* Round a value to BF16 the way the GPU does: first to FP32 (nearest even),
 * then to the top 16 bits of the FP32 pattern (nearest even). */
static double bf16(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return v;  /* inf / nan unchanged */
    u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

int orc_bf16_round(const double* in, uint32_t n, double* out)
{
    for (uint32_t i = 0; i < n; ++i) out[i] = bf16(in[i]);
    return 0;
}

int orc_mlp_encode(const float* pos, const float* nrm, uint32_t n, const float* lo, const float* hi, double* out)
{
    for (uint32_t i = 0; i < n; ++i) {
        double v[6];
        /* the normalised position is formed in FP32, as the inputs are */
        for (int a = 0; a < 3; ++a) {
            float num = pos[3 * i + a] - lo[a];
            float den = hi[a] - lo[a];
            v[a] = (double)(num / den);
        }
        for (int a = 0; a < 3; ++a) v[3 + a] = nrm[3 * i + a];
        for (int c = 0; c < 6; ++c)
            for (int k = 0; k < 12; ++k) {
                double arg = PI * ldexp(v[c], k);
                out[(size_t)i * IN + 24 * c + 2 * k] = sin(arg);
                out[(size_t)i * IN + 24 * c + 2 * k + 1] = cos(arg);
            }
    }
    return 0;
}

typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
} params_view;

static params_view view(const double* p)
{
    params_view v;
    v.W1 = p;
    v.b1 = v.W1 + H * IN;
    v.W2 = v.b1 + H;
    v.b2 = v.W2 + H * H;
    v.W3 = v.b2 + H;
    v.b3 = v.W3 + H * H;
    v.W4 = v.b3 + H;
    v.b4 = v.W4 + OUT * H;
    return v;
}

/* y[o] = b[o] + sum_i W[o][i] x[i] */
static void dense(const double* W, const double* b, const double* x, int nin, int nout, double* y)
{
    for (int o = 0; o < nout; ++o) {
        double acc = 0.0;
        for (int i = 0; i < nin; ++i) acc += W[o * nin + i] * x[i];
        y[o] = acc + b[o];
    }
}

/* One sample forward pass; keeps what the backward pass needs. */
typedef struct {
    double x[IN];
    double h1[H], a1[H];
    double h2[H], a2[H];
    double h3[H], a3[H];
    double z[OUT], q[OUT];
} trace;

static void forward_one(const double* pw, const double* p, const double* xin, int use_bf16, trace* t)
{
    /* pw: the weights as used (BF16-rounded in bf16 mode); p: the parameters
     * as stored, from which the biases are taken at full precision (the GPU
     * adds them to FP32 sums) */
    params_view v = view(pw);
    params_view vb = view(p);
    for (int i = 0; i < IN; ++i) t->x[i] = use_bf16 ? bf16(xin[i]) : xin[i];
    dense(v.W1, vb.b1, t->x, IN, H, t->h1);
    for (int j = 0; j < H; ++j) {
        double r = t->h1[j] > 0.0 ? t->h1[j] : 0.0;
        t->a1[j] = use_bf16 ? bf16(r) : r;
    }
    dense(v.W2, vb.b2, t->a1, H, H, t->h2);
    for (int j = 0; j < H; ++j) {
        double r = t->h2[j] > 0.0 ? t->h2[j] : 0.0;
        t->a2[j] = use_bf16 ? bf16(r) : r;
    }
    dense(v.W3, vb.b3, t->a2, H, H, t->h3);
    for (int j = 0; j < H; ++j) {
        double r = t->h3[j] > 0.0 ? t->h3[j] : 0.0;
        t->a3[j] = use_bf16 ? bf16(r) : r;
    }
    dense(v.W4, vb.b4, t->a3, H, OUT, t->z);
    /* softmax */
    double zmax = t->z[0];
    for (int k = 1; k < OUT; ++k) zmax = t->z[k] > zmax ? t->z[k] : zmax;
    double s = 0.0;
    for (int k = 0; k < OUT; ++k) {
        t->q[k] = exp(t->z[k] - zmax);
        s += t->q[k];
    }
    for (int k = 0; k < OUT; ++k) t->q[k] /= s;
}

/* The weights as the network uses them: rounded to BF16 in bf16 mode. */
static double* used_weights(const double* p, int use_bf16)
{
    double* pw = (double*)malloc(sizeof(double) * NPARAM);
    if (!pw) return NULL;
    for (int i = 0; i < NPARAM; ++i) pw[i] = use_bf16 ? bf16(p[i]) : p[i];
    return pw;
}

/* logits (n x 64) and softmax probabilities (n x 64) */
int orc_mlp_forward(const double* params, const double* x, uint32_t n, int use_bf16, double* logits, double* probs)
{
    trace* t = (trace*)malloc(sizeof(trace));
    double* pw = used_weights(params, use_bf16);
    if (!t || !pw) {
        free(t);
        free(pw);
        return -2;
    }
    for (uint32_t i = 0; i < n; ++i) {
        forward_one(pw, params, x + (size_t)i * IN, use_bf16, t);
        if (logits) memcpy(logits + (size_t)i * OUT, t->z, sizeof(t->z));
        if (probs) memcpy(probs + (size_t)i * OUT, t->q, sizeof(t->q));
    }
    free(t);
    free(pw);
    return 0;
}

/* Loss and its gradient with respect to every parameter (same layout).
 * The per-tuple output gradient is w_i (q_i - e_{k_i}); it and the
 * back-propagated gradients are what the bf16 mode rounds; the sums over the
 * batch are divided by sum_i w_i at the end (all zero when that sum is 0). */
int orc_mlp_loss_grad(const double* params, const double* x, const uint32_t* node, const double* w, uint32_t n,
                      int use_bf16, double* loss, double* grad)
{
    double* pw = used_weights(params, use_bf16);
    if (!pw) return -2;
    params_view v = view(pw);
    memset(grad, 0, sizeof(double) * NPARAM);
    double* gW1 = grad;
    double* gb1 = gW1 + H * IN;
    double* gW2 = gb1 + H;
    double* gb2 = gW2 + H * H;
    double* gW3 = gb2 + H;
    double* gb3 = gW3 + H * H;
    double* gW4 = gb3 + H;
    double* gb4 = gW4 + OUT * H;
    double wsum = 0.0;
    for (uint32_t i = 0; i < n; ++i) wsum += w[i];
    double L = 0.0;
    trace* t = (trace*)malloc(sizeof(trace));
    if (!t) {
        free(pw);
        return -2;
    }
    for (uint32_t i = 0; i < n; ++i) {
        if (node[i] >= OUT) {
            free(t);
            free(pw);
            return -1;
        }
        forward_one(pw, params, x + (size_t)i * IN, use_bf16, t);
        L -= w[i] * log(t->q[node[i]] > 0.0 ? t->q[node[i]] : 1e-300);
        double g4[OUT], d3[H], d2[H], d1[H];
        for (int k = 0; k < OUT; ++k) {
            double g = w[i] * (t->q[k] - (k == (int)node[i] ? 1.0 : 0.0));
            g4[k] = use_bf16 ? bf16(g) : g;
        }
        for (int k = 0; k < OUT; ++k) {
            gb4[k] += g4[k];
            for (int j = 0; j < H; ++j) gW4[k * H + j] += g4[k] * t->a3[j];
        }
        for (int j = 0; j < H; ++j) {
            double acc = 0.0;
            for (int k = 0; k < OUT; ++k) acc += g4[k] * v.W4[k * H + j];
            double d = t->h3[j] > 0.0 ? acc : 0.0;
            d3[j] = use_bf16 ? bf16(d) : d;
        }
        for (int o = 0; o < H; ++o) {
            gb3[o] += d3[o];
            for (int j = 0; j < H; ++j) gW3[o * H + j] += d3[o] * t->a2[j];
        }
        for (int j = 0; j < H; ++j) {
            double acc = 0.0;
            for (int o = 0; o < H; ++o) acc += d3[o] * v.W3[o * H + j];
            double d = t->h2[j] > 0.0 ? acc : 0.0;
            d2[j] = use_bf16 ? bf16(d) : d;
        }
        for (int o = 0; o < H; ++o) {
            gb2[o] += d2[o];
            for (int j = 0; j < H; ++j) gW2[o * H + j] += d2[o] * t->a1[j];
        }
        for (int j = 0; j < H; ++j) {
            double acc = 0.0;
            for (int o = 0; o < H; ++o) acc += d2[o] * v.W2[o * H + j];
            double d = t->h1[j] > 0.0 ? acc : 0.0;
            d1[j] = use_bf16 ? bf16(d) : d;
        }
        for (int o = 0; o < H; ++o) {
            gb1[o] += d1[o];
            for (int j = 0; j < IN; ++j) gW1[o * IN + j] += d1[o] * t->x[j];
        }
    }
    free(t);
    free(pw);
    double inv = wsum > 0.0 ? 1.0 / wsum : 0.0;
    for (int i = 0; i < NPARAM; ++i) grad[i] *= inv;
    if (loss) *loss = L * inv;
    return 0;
}

/* One Adam step (Kingma and Ba, 2015) on FP64 parameters. */
int orc_mlp_adam(double* params, double* m, double* v, const double* grad, uint32_t n, uint32_t step, double lr,
                 double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)step);
    double c2 = 1.0 - pow(beta2, (double)step);
    for (uint32_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        params[i] -= lr * mh / (sqrt(vh) + eps);
    }
    return 0;
}

/* Training order (not fixed by the paper; a reading): batch position i of
 * epoch e takes tuple pi_e(i), where pi_e is a keyed pseudo-random
 * permutation of 0..n-1 that needs no sort.  pi_e is a balanced Feistel
 * network of eight rounds on 2h-bit words (h the smallest with 4^h >= n, at
 * least 1; Luby and Rackoff 1988): round r maps the halves (L, R) to
 * (R, L xor (F(R xor k_r) mod 2^h)), with F the 32-bit finaliser of
 * MurmurHash3 (Appleby) and k_{4j+w} word w of Philox at counter
 * (j, e, 0, scene << 16 | 2), j = 0, 1.  (Four rounds leave neighbouring
 * positions visibly correlated when the halves are a few bits wide.)  The
 * network permutes 0..4^h-1; a value of n or more is sent through it again
 * until one falls below n (cycle walking, Black and Rogaway 2002), which
 * keeps the map a permutation of 0..n-1. */
int orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, uint32_t n);

static uint32_t murmur3_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

static uint32_t feistel_rounds(uint32_t x, uint32_t h, const uint32_t k[8])
{
    const uint32_t mask = (uint32_t)((1ull << h) - 1ull);
    uint32_t left = (uint32_t)((uint64_t)x >> h), right = x & mask;
    for (int r = 0; r < 8; ++r) {
        uint32_t next = left ^ (murmur3_fmix32(right ^ k[r]) & mask);
        left = right;
        right = next;
    }
    return (uint32_t)(((uint64_t)left << h) | right);
}

int orc_mlp_shuffle(uint32_t n, uint32_t epoch, uint32_t scene_id, uint64_t seed, uint32_t* perm)
{
    uint32_t h = 1;
    while ((1ull << (2u * h)) < (uint64_t)n) ++h;
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32)}, k[8];
    for (uint32_t j = 0; j < 2; ++j) {
        uint32_t ctr[4] = {j, epoch, 0u, (scene_id << 16) | 2u};
        orc_philox(ctr, key, k + 4 * j, 1);
    }
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t x = i;
        do
            x = feistel_rounds(x, h, k);
        while (x >= n);
        perm[i] = x;
    }
    return 0;
}

/* Minibatch training over logged tuples (point id, fixed-cut node, weight):
 * for each epoch the shuffled order is cut into batches of up to B tuples
 * (the last one may be short); each batch takes one Adam step.  xall holds
 * the encoded inputs of every point (rows of 144).  step is the Adam step
 * count so far; the new count is returned through it. */
int orc_mlp_train(double* params, double* m, double* v, uint32_t* step, const double* xall, uint32_t npts,
                  const uint32_t* pid, const uint32_t* node, const double* w, uint32_t n, uint32_t epochs,
                  uint32_t B, double lr, double beta1, double beta2, double eps, uint32_t scene_id, uint64_t seed,
                  int use_bf16, double* last_loss)
{
    if (B == 0) return -1;
    for (uint32_t i = 0; i < n; ++i)
        if (pid[i] >= npts || node[i] >= OUT) return -1;
    uint32_t* perm = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1u));
    double* xb = (double*)malloc(sizeof(double) * IN * (size_t)B);
    uint32_t* nb = (uint32_t*)malloc(sizeof(uint32_t) * B);
    double* wb = (double*)malloc(sizeof(double) * B);
    double* g = (double*)malloc(sizeof(double) * NPARAM);
    int rc = (perm && xb && nb && wb && g) ? 0 : -2;
    for (uint32_t e = 0; rc == 0 && e < epochs; ++e) {
        rc = orc_mlp_shuffle(n, e, scene_id, seed, perm);
        for (uint32_t b0 = 0; rc == 0 && b0 < n; b0 += B) {
            uint32_t nbat = n - b0 < B ? n - b0 : B;
            for (uint32_t j = 0; j < nbat; ++j) {
                uint32_t t = perm[b0 + j];
                memcpy(xb + (size_t)j * IN, xall + (size_t)pid[t] * IN, sizeof(double) * IN);
                nb[j] = node[t];
                wb[j] = w[t];
            }
            double L = 0.0;
            rc = orc_mlp_loss_grad(params, xb, nb, wb, nbat, use_bf16, &L, g);
            if (rc == 0) {
                *step += 1u;
                orc_mlp_adam(params, m, v, g, NPARAM, *step, lr, beta1, beta2, eps);
                if (last_loss) *last_loss = L;
            }
        }
    }
    free(perm);
    free(xb);
    free(nb);
    free(wb);
    free(g);
    return rc;
}
