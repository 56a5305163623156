// The learned proposal: a 144 -> 64 -> 64 -> 64 -> 64 MLP (ReLU hidden
// layers, softmax output) from a point's position and normal to a
// distribution over the nodes of a fixed 64-node breadth-first cut.  It is
// mixed with the cell's cut distribution when sampling, so the estimator
// stays unbiased, and trained on the (point, node, contribution / density)
// records the frames log, by minimising the weighted cross-entropy
// -sum_i w_i log q_i[k_i] / sum_i w_i (the one-sample form of the KL
// divergence from the contribution-proportional target) with Adam.
//
// Arithmetic: BF16 operands on the matrix cores with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16), FP32 biases, softmax and optimizer.
//
// MFMA operand layout (one wave, lane l = 16 g + i):
//   A (16 x 32): lane holds A[i][8 g + e], e = 0..7
//   B (32 x 16): lane holds B[8 g + e][i]
//   D (16 x 16): lane holds D[4 g + r][i], r = 0..3
// A layer computes its output transposed, H^T = W X^T: A is a 16-row tile
// of W, B the inputs of 16 points, D the tile's 16 units for those points.
// The D registers of two neighbouring tiles are exactly the 8 values one
// lane contributes to the next layer's B operand if the next layer's
// weights are stored with their input units in the matching order
// (hidden_pos below), so activations never leave registers.
#include "mlp_internal.h"

namespace rlc {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;
constexpr uint32_t kIn = 144, kH = 64;
constexpr uint32_t kNP = kMlpParams;
// flat parameter layout: W1 [64][144], b1, W2 [64][64], b2, W3, b3, W4, b4
constexpr uint32_t oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
                   ob3 = oW3 + kH * kH, oW4 = ob3 + kH, ob4 = oW4 + kH * kH;
static_assert(ob4 + kH == kNP, "parameter count");
// fragment regions, in 16-byte vectors: forward operands of layers 1-4 (A =
// W tile), then transposed operands of layers 2-4 (A = W^T tile) used to
// back-propagate; [tile][k-block][lane]
constexpr uint32_t fF1 = 0, fF2 = 1280, fF3 = 1792, fF4 = 2304, fT2 = 2816, fT3 = 3328, fT4 = 3840;
static_assert(fT4 + 512 == kMlpFragVecs, "fragment count");
constexpr uint32_t kFwdVecs = fT2;

__device__ __forceinline__ uint16_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Eight floats to BF16 by the hardware's conversion (v_cvt_pk_bf16_f32,
// two per instruction, round to nearest even like bf16_bits).
__device__ __forceinline__ bf16x8 pack8(const float* v) {
    bf16x8 b;
#pragma unroll
    for (int e = 0; e < 8; ++e) b[e] = (__bf16)v[e];
    return b;
}

__device__ __forceinline__ uint16_t elem(bf16x8 v, int e) { return __builtin_bit_cast(u16x8, v)[e]; }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Slot of hidden unit j in the B operand built from accumulator registers:
// k-block kb, lane group g, element e, with j = 32 kb + 16 (e / 4) + 4 g + e % 4.
__device__ __forceinline__ void hidden_pos(uint32_t j, uint32_t& kb, uint32_t& g, uint32_t& e) {
    kb = j >> 5;
    const uint32_t r = j & 31u;
    g = (r & 15u) >> 2;
    e = 4u * (r >> 4) + (r & 3u);
}

// Fragment element of weight W_L[o][j] in the forward operands, and (layers
// 2-4) in the transposed ones.
__device__ __forceinline__ uint32_t frag_fwd(uint32_t layer, uint32_t o, uint32_t j) {
    const uint32_t t = o >> 4, i = o & 15u;
    if (layer == 1u) {
        const uint32_t kb = j >> 5, g = (j & 31u) >> 3, e = j & 7u;
        return ((fF1 + (t * 5u + kb) * 64u + 16u * g + i) << 3) + e;
    }
    uint32_t kb, g, e;
    hidden_pos(j, kb, g, e);
    const uint32_t base = layer == 2u ? fF2 : (layer == 3u ? fF3 : fF4);
    return ((base + (t * 2u + kb) * 64u + 16u * g + i) << 3) + e;
}

__device__ __forceinline__ uint32_t frag_tr(uint32_t layer, uint32_t o, uint32_t j) {
    const uint32_t t = j >> 4, i = j & 15u;
    uint32_t kb, g, e;
    hidden_pos(o, kb, g, e);
    const uint32_t base = layer == 2u ? fT2 : (layer == 3u ? fT3 : fT4);
    return ((base + (t * 2u + kb) * 64u + 16u * g + i) << 3) + e;
}

// Parameter p -> (layer, o, j) for weights; false for a bias.
__device__ __forceinline__ bool weight_of(uint32_t p, uint32_t& layer, uint32_t& o, uint32_t& j) {
    if (p < ob1) {
        layer = 1u;
        o = p / kIn;
        j = p % kIn;
        return true;
    }
    const uint32_t offs[3] = {oW2, oW3, oW4};
#pragma unroll
    for (uint32_t L = 0; L < 3; ++L)
        if (p >= offs[L] && p < offs[L] + kH * kH) {
            layer = L + 2u;
            o = (p - offs[L]) >> 6;
            j = (p - offs[L]) & 63u;
            return true;
        }
    return false;
}

__device__ __forceinline__ void write_frag(uint16_t* frag, uint32_t p, float val) {
    uint32_t layer, o, j;
    if (!weight_of(p, layer, o, j)) return;
    const uint16_t b = bf16_bits(val);
    frag[frag_fwd(layer, o, j)] = b;
    if (layer > 1u) frag[frag_tr(layer, o, j)] = b;
}

// The inputs a lane supplies to layer 1 for its point: for k-block kb the 8
// encoded values 32 kb + 8 g .. + 7 (value 24 c + 2 k + {0, 1} is sin / cos
// of 2^k pi v_c); indices from 144 on are zero padding.
__device__ __forceinline__ void encode_b(const float v[6], uint32_t g, bf16x8 xb[5]) {
#pragma unroll
    for (uint32_t kb = 0; kb < 5u; ++kb) {
        const uint32_t base = 32u * kb + 8u * g;
        float val[8];
        if (base < kIn) {
            const uint32_t c = base / 24u, m = (base % 24u) >> 3;
#pragma unroll
            for (uint32_t e2 = 0; e2 < 4u; ++e2) {
                const float ph = ldexpf(v[c], (int)(4u * m + e2));
                val[2 * e2] = sinpif(ph);
                val[2 * e2 + 1] = cospif(ph);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) val[e] = 0.0f;
        }
        xb[kb] = pack8(val);
    }
}

__device__ __forceinline__ void point_inputs(const MlpEncode& enc, const float* pos, const float* nrm, uint32_t p,
                                             float v[6]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float num = pos[3 * (size_t)p + a] - enc.lo[a];
        v[a] = num / enc.ext[a];
        v[3 + a] = nrm[3 * (size_t)p + a];
    }
}

// One dense layer for 16 points: out[t] = W tile t . B + bias (FP32).
template <int KB>
__device__ __forceinline__ void dense(const bf16x8* __restrict__ frag, const bf16x8 (&b)[KB],
                                      const float* __restrict__ bias, uint32_t lane, f32x4 (&out)[4]) {
    const uint32_t g = lane >> 4;
#pragma unroll
    for (uint32_t t = 0; t < 4u; ++t) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) acc = mfma(frag[(t * KB + kb) * 64u + lane], b[kb], acc);
#pragma unroll
        for (uint32_t r = 0; r < 4u; ++r) out[t][r] = acc[r] + bias[16u * t + 4u * g + r];
    }
}

// ReLU of two tiles' registers into the next layer's B operand (BF16).
__device__ __forceinline__ void relu_to_b(const f32x4 (&h)[4], bf16x8 (&b)[2]) {
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        float val[8];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            val[r] = h[2 * kb][r] > 0.0f ? h[2 * kb][r] : 0.0f;
            val[4 + r] = h[2 * kb + 1][r] > 0.0f ? h[2 * kb + 1][r] : 0.0f;
        }
        b[kb] = pack8(val);
    }
}

struct Fwd {
    bf16x8 x[5];
    f32x4 h1[4], h2[4], h3[4], z[4];
    bf16x8 a1[2], a2[2], a3[2];
};

// The layers for 16 points whose encoded inputs are in f.x.
__device__ __forceinline__ void forward16(const bf16x8* __restrict__ frag, const float* __restrict__ master,
                                          uint32_t lane, Fwd& f) {
    dense<5>(frag + fF1, f.x, master + ob1, lane, f.h1);
    relu_to_b(f.h1, f.a1);
    dense<2>(frag + fF2, f.a1, master + ob2, lane, f.h2);
    relu_to_b(f.h2, f.a2);
    dense<2>(frag + fF3, f.a2, master + ob3, lane, f.h3);
    relu_to_b(f.h3, f.a3);
    dense<2>(frag + fF4, f.a3, master + ob4, lane, f.z);
}

// Softmax over a point's 64 logits, which sit in the 4 lanes i, i+16, i+32,
// i+48 (16 each).  Returns the probabilities in place of the logits and the
// log of the normaliser relative to the max.
__device__ __forceinline__ void softmax16(f32x4 (&z)[4], float& zmax, float& log_s) {
    float m = z[0][0];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) m = fmaxf(m, z[t][r]);
    m = fmaxf(m, __shfl_xor(m, 16, 64));
    m = fmaxf(m, __shfl_xor(m, 32, 64));
    float s = 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            z[t][r] = expf(z[t][r] - m);
            s += z[t][r];
        }
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) z[t][r] = z[t][r] / s;
    zmax = m;
    log_s = logf(s);
}

// ---------------------------------------------------------------------------
// Inference: per point, the inclusive running sums of the 64 probabilities
// (and optionally the logits).  Blocks stage the forward operands in LDS and
// walk groups of 16 points, one group per wave per round.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_mlp_forward(const bf16x8* __restrict__ frag,
                                                        const float* __restrict__ master, MlpEncode enc,
                                                        const float* __restrict__ pos,
                                                        const float* __restrict__ nrm, uint32_t P,
                                                        float* __restrict__ cdf, float* __restrict__ logits) {
    __shared__ bf16x8 s_frag[kFwdVecs];
    __shared__ float s_q[4][16][65];
    for (uint32_t j = threadIdx.x; j < kFwdVecs; j += kBlock) s_frag[j] = frag[j];
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, i16 = lane & 15u, g = lane >> 4;
    const uint32_t ngroups = (P + 15u) >> 4;
    for (uint32_t base = blockIdx.x * 4u; base < ngroups; base += gridDim.x * 4u) {
        const uint32_t grp = base + wave;
        const uint32_t p = grp * 16u + i16;
        const bool valid = grp < ngroups && p < P;
        float v[6];
        point_inputs(enc, pos, nrm, valid ? p : 0u, v);
        Fwd f;
        encode_b(v, g, f.x);
        forward16(s_frag, master, lane, f);
        if (valid && logits) {
#pragma unroll
            for (uint32_t t = 0; t < 4u; ++t)
                *reinterpret_cast<float4*>(logits + (size_t)p * 64u + 16u * t + 4u * g) =
                    make_float4(f.z[t][0], f.z[t][1], f.z[t][2], f.z[t][3]);
        }
        float zmax, log_s;
        softmax16(f.z, zmax, log_s);
#pragma unroll
        for (uint32_t t = 0; t < 4u; ++t)
#pragma unroll
            for (uint32_t r = 0; r < 4u; ++r) s_q[wave][i16][16u * t + 4u * g + r] = f.z[t][r];
        __syncthreads();
        if (valid && g == 0u && cdf) {
            float acc = 0.0f;
            float* row = cdf + (size_t)p * 64u;
            for (uint32_t k = 0; k < 64u; k += 4u) {
                float4 o;
                acc = acc + s_q[wave][i16][k];
                o.x = acc;
                acc = acc + s_q[wave][i16][k + 1u];
                o.y = acc;
                acc = acc + s_q[wave][i16][k + 2u];
                o.z = acc;
                acc = acc + s_q[wave][i16][k + 3u];
                o.w = acc;
                *reinterpret_cast<float4*>(row + k) = o;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Training: forward and backward of kTrainTuples tuples per block (16 per
// wave), and the block's share of the weight gradient, sum over its tuples
// of G_L A_{L-1}^T, staged through LDS one layer at a time as MFMA
// contractions over the block's tuples.  Writes one row of partial sums
// (all parameters), and the block's sum of weights and of weighted losses;
// the reduction over blocks is done in a fixed order by k_mlp_reduce.
// Eight waves (128 tuples) per block: measured against 64 and 256 tuples
// per block (the partial rows halve with each doubling, but fewer blocks
// hold fewer waves in flight for the latency of the layer chain).  Between
// the layers only what the backward pass needs stays in registers: the BF16
// activations and, for the ReLU derivative, one bit per pre-activation.
// ---------------------------------------------------------------------------
constexpr uint32_t kTrainWaves = kMlpTuplesPerBlock / 16u;
static_assert(kTrainWaves >= 4u && kTrainWaves <= 16u, "4 to 16 waves per training block");
constexpr uint32_t kTrainThreads = kTrainWaves * 64u;
constexpr uint32_t kTrainTuples = kTrainWaves * 16u;
constexpr uint32_t kLdsT = kTrainTuples + 8u;  // LDS row stride (BF16) of the staging tiles

__device__ __forceinline__ void stage_hidden(uint16_t* __restrict__ s, const bf16x8 (&b)[2], uint32_t g,
                                             uint32_t col) {
#pragma unroll
    for (uint32_t kb = 0; kb < 2u; ++kb)
#pragma unroll
        for (uint32_t e = 0; e < 8u; ++e) {
            const uint32_t j = 32u * kb + 16u * (e >> 2) + 4u * g + (e & 3u);
            s[j * kLdsT + col] = elem(b[kb], (int)e);
        }
}

// gW tile (to, tj) over the block's tuples, written to the partial row.
__device__ __forceinline__ void wgrad_tile(const uint16_t* __restrict__ sG, const uint16_t* __restrict__ sA,
                                           uint32_t to, uint32_t tj, uint32_t nin, uint32_t lane,
                                           float* __restrict__ prow) {
    const uint32_t i16 = lane & 15u, g = lane >> 4;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (uint32_t kb = 0; kb < kTrainTuples / 32u; ++kb) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(sG + (16u * to + i16) * kLdsT + 32u * kb + 8u * g);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(sA + (16u * tj + i16) * kLdsT + 32u * kb + 8u * g);
        acc = mfma(a, b, acc);
    }
#pragma unroll
    for (uint32_t r = 0; r < 4u; ++r) prow[(16u * to + 4u * g + r) * nin + 16u * tj + i16] = acc[r];
}

// Bias gradient of one layer: row j of sG summed over the block's tuples,
// four threads per row, each over a quarter of the columns, the quarters
// added in order (the four are neighbouring lanes).
__device__ __forceinline__ void bias_grad(const uint16_t* __restrict__ sG, float* __restrict__ dst) {
    if (threadIdx.x >= 4u * kH) return;
    const uint32_t row = threadIdx.x >> 2, q = threadIdx.x & 3u;
    constexpr uint32_t kQ = kTrainTuples / 4u;
    float sum = 0.0f;
    for (uint32_t c = 0; c < kQ; ++c) sum += bf16_val(sG[row * kLdsT + q * kQ + c]);
    const float s1 = __shfl(sum, (int)((threadIdx.x & 63u) | 1u), 64);
    const float s2 = __shfl(sum, (int)((threadIdx.x & 63u) | 2u), 64);
    const float s3 = __shfl(sum, (int)((threadIdx.x & 63u) | 3u), 64);
    if (q == 0u) dst[row] = ((sum + s1) + s2) + s3;
}

// One dense layer, then the ReLU into the next layer's B operand, keeping
// one bit per pre-activation (bit 4 t + r: tile t, register r is > 0).
template <int KB>
__device__ __forceinline__ uint32_t hidden_layer(const bf16x8* __restrict__ frag, const bf16x8 (&b)[KB],
                                                 const float* __restrict__ bias, uint32_t lane,
                                                 bf16x8 (&out)[2]) {
    f32x4 h[4];
    dense<KB>(frag, b, bias, lane, h);
    uint32_t mask = 0;
#pragma unroll
    for (uint32_t t = 0; t < 4u; ++t)
#pragma unroll
        for (uint32_t r = 0; r < 4u; ++r)
            if (h[t][r] > 0.0f) mask |= 1u << (4u * t + r);
    relu_to_b(h, out);
    return mask;
}

// The work of training block blk (its kTrainTuples tuples of the n given):
// forward, backward, and its row of partial sums.
__device__ __forceinline__ void train_block(uint32_t blk, const bf16x8* frag, const float* master,
                                            const MlpEncode& enc, const float* __restrict__ pos,
                                            const float* __restrict__ nrm, uint32_t P,
                                            const bf16x8* __restrict__ xenc, const MlpOrder& ord, uint32_t base,
                                            const uint32_t* __restrict__ pid, const uint32_t* __restrict__ node,
                                            const float* __restrict__ w, uint32_t n, float* partial, float* part_w,
                                            float* part_loss, uint32_t* err) {
    __shared__ __attribute__((aligned(16))) uint16_t sG[kH * kLdsT];
    __shared__ __attribute__((aligned(16))) uint16_t sA[kIn * kLdsT];
    __shared__ float s_w[kTrainTuples], s_l[kTrainTuples];
    // the block's copy of every weight operand (forward and transposed) and
    // of the biases: each wave reads its operands from LDS instead of
    // fetching the same 70 KB from L2
    __shared__ bf16x8 s_frag[kMlpFragVecs];
    __shared__ float s_bias[4u * kH];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, i16 = lane & 15u, g = lane >> 4;
    const uint32_t col = wave * 16u + i16;
    const uint32_t tb = blk * kTrainTuples + col;
    // the staging loads are issued first; the tuple's place in the epoch
    // order is computed and its record fetched while they are in flight
    constexpr uint32_t kPer = (kMlpFragVecs + kTrainThreads - 1u) / kTrainThreads;
    bf16x8 v[kPer];
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t j = threadIdx.x + k * kTrainThreads;
        if (j < kMlpFragVecs) v[k] = frag[j];
    }
    float bv = 0.0f;
    if (threadIdx.x < 4u * kH) {
        const uint32_t L = threadIdx.x / kH;
        bv = master[(L == 0u ? ob1 : (L == 1u ? ob2 : (L == 2u ? ob3 : ob4))) + threadIdx.x % kH];
    }
    uint32_t pt = 0, nd = 0;
    float wt = 0.0f;
    if (tb < n) {
        const uint32_t t = ord.n ? mlp_order_at(ord, base + tb) : tb;
        pt = pid[t];
        nd = node[t];
        wt = w[t];
    }
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t j = threadIdx.x + k * kTrainThreads;
        if (j < kMlpFragVecs) s_frag[j] = v[k];
    }
    if (threadIdx.x < 4u * kH) s_bias[threadIdx.x] = bv;
    if (tb < n && (pt >= P || nd >= 64u || !(wt >= 0.0f && wt <= 3.402823466e38f))) {
        if (g == 0u) atomicOr(err, RLC_DERR_INPUT);
        pt = 0;
        nd = 0;
        wt = 0.0f;
    }
    // the point's encoded inputs (computed once per call, or here)
    auto load_x = [&](bf16x8 (&x)[5]) {
        if (xenc) {
#pragma unroll
            for (uint32_t kb = 0; kb < 5u; ++kb) x[kb] = xenc[((size_t)pt * 5u + kb) * 4u + g];
        } else {
            float v[6];
            point_inputs(enc, pos, nrm, pt, v);
            encode_b(v, g, x);
        }
    };
    bf16x8 a1[2], a2[2], a3[2];
    uint32_t m1, m2, m3;
    f32x4 z[4];
    // the encoded inputs stay in registers for layer 1's weight gradient
    bf16x8 x[5];
    load_x(x);
    __syncthreads();  // the staged operands
    m1 = hidden_layer<5>(s_frag + fF1, x, s_bias, lane, a1);
    m2 = hidden_layer<2>(s_frag + fF2, a1, s_bias + kH, lane, a2);
    m3 = hidden_layer<2>(s_frag + fF3, a2, s_bias + 2u * kH, lane, a3);
    dense<2>(s_frag + fF4, a3, s_bias + 3u * kH, lane, z);
    // the target's logit, from the lane that holds it (before the softmax
    // replaces the logits by probabilities)
    const uint32_t tn = nd >> 4, gn = (nd & 15u) >> 2, rn = nd & 3u;
    float zn = 0.0f;
#pragma unroll
    for (uint32_t t = 0; t < 4u; ++t)
#pragma unroll
        for (uint32_t r = 0; r < 4u; ++r)
            if (t == tn && r == rn) zn = z[t][r];
    float zmax, log_s;
    softmax16(z, zmax, log_s);
    // loss term -w log q[node]
    if (g == gn) {
        s_l[col] = -(wt * ((zn - zmax) - log_s));
        s_w[col] = wt;
    }
    // output gradient w (q - e_node)
    bf16x8 gB[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        float val[8];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t u0 = 16u * (2u * kb) + 4u * g + r, u1 = 16u * (2u * kb + 1u) + 4u * g + r;
            val[r] = wt * (z[2 * kb][r] - (u0 == nd ? 1.0f : 0.0f));
            val[4 + r] = wt * (z[2 * kb + 1][r] - (u1 == nd ? 1.0f : 0.0f));
        }
        gB[kb] = pack8(val);
    }
    // back-propagation through the transposed operands, with the ReLU bits
    auto back = [&](const bf16x8* __restrict__ fr, const bf16x8 (&gin)[2], uint32_t mask, bf16x8 (&gout)[2]) {
        f32x4 d[4];
#pragma unroll
        for (uint32_t t = 0; t < 4u; ++t) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (uint32_t kb = 0; kb < 2u; ++kb) acc = mfma(fr[(t * 2u + kb) * 64u + lane], gin[kb], acc);
#pragma unroll
            for (uint32_t r = 0; r < 4u; ++r) d[t][r] = (mask >> (4u * t + r)) & 1u ? acc[r] : 0.0f;
        }
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            float val[8];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                val[r] = d[2 * kb][r];
                val[4 + r] = d[2 * kb + 1][r];
            }
            gout[kb] = pack8(val);
        }
    };
    float* prow = partial + (size_t)blk * kNP;
    // layers 4, 3, 2, each in turn: G_L and the previous activations staged
    // in LDS, G_{L-1} propagated from G_L, then the layer's weight gradient
    // (16 tiles over the waves) and bias gradient; a layer's operands are not
    // needed once staged
    auto layer_grad = [&](const bf16x8 (&act)[2], const bf16x8* __restrict__ fr_t, uint32_t mask, uint32_t ow_,
                          uint32_t ob_) {
        stage_hidden(sG, gB, g, col);
        stage_hidden(sA, act, g, col);
        bf16x8 gn2[2];
        back(fr_t, gB, mask, gn2);
        gB[0] = gn2[0];
        gB[1] = gn2[1];
        __syncthreads();
        for (uint32_t tile = wave; tile < 16u; tile += kTrainWaves)  // 4 output x 4 input tiles
            wgrad_tile(sG, sA, tile >> 2, tile & 3u, kH, lane, prow + ow_);
        bias_grad(sG, prow + ob_);
        __syncthreads();
    };
    layer_grad(a3, s_frag + fT4, m3, oW4, ob4);
    layer_grad(a2, s_frag + fT3, m2, oW3, ob3);
    layer_grad(a1, s_frag + fT2, m1, oW2, ob2);
    // layer 1: G_1 against the encoded inputs (144 rows): 36 tiles
    stage_hidden(sG, gB, g, col);
#pragma unroll
    for (uint32_t kb = 0; kb < 5u; ++kb)
#pragma unroll
        for (uint32_t e = 0; e < 8u; ++e) {
            const uint32_t j = 32u * kb + 8u * g + e;
            if (j < kIn) sA[j * kLdsT + col] = elem(x[kb], (int)e);
        }
    __syncthreads();
    for (uint32_t tile = wave; tile < 36u; tile += kTrainWaves)  // 4 output x 9 input tiles
        wgrad_tile(sG, sA, tile / 9u, tile % 9u, kIn, lane, prow + oW1);
    bias_grad(sG, prow + ob1);
    // the block's sums of weights and of weighted losses, by wave 0 in a
    // fixed order: each lane adds its kTrainTuples / 64 entries, then a
    // butterfly across the lanes
    if (wave == 0u) {
        float sw = 0.0f, sl = 0.0f;
#pragma unroll
        for (uint32_t c = lane; c < kTrainTuples; c += 64u) {
            sw += s_w[c];
            sl += s_l[c];
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            sw += __shfl_xor(sw, off, 64);
            sl += __shfl_xor(sl, off, 64);
        }
        if (lane == 0u) {
            part_w[blk] = sw;
            part_loss[blk] = sl;
        }
    }
}

__global__ void __launch_bounds__(kTrainThreads) k_mlp_fwd_bwd(const bf16x8* __restrict__ frag,
                                                               const float* __restrict__ master, MlpEncode enc,
                                                               const float* __restrict__ pos,
                                                               const float* __restrict__ nrm, uint32_t P,
                                                               const bf16x8* __restrict__ xenc, MlpOrder ord,
                                                               uint32_t base, const uint32_t* __restrict__ pid,
                                                               const uint32_t* __restrict__ node,
                                                               const float* __restrict__ w, uint32_t n,
                                                               float* __restrict__ partial,
                                                               float* __restrict__ part_w,
                                                               float* __restrict__ part_loss,
                                                               uint32_t* __restrict__ err) {
    train_block(blockIdx.x, frag, master, enc, pos, nrm, P, xenc, ord, base, pid, node, w, n, partial, part_w,
                part_loss, err);
}

constexpr uint32_t kRedCols = 32, kRedGroups = kBlock / kRedCols;

// Column p of the blocks' partial rows, the rows of group grp (grp, grp +
// kRedGroups, ...) added in that order; the loads of a run of 32 (then 8)
// rows are issued before their additions.
__device__ __forceinline__ float column_sum(const float* partial, uint32_t p, uint32_t grp, uint32_t nblocks) {
    float acc = 0.0f;
    uint32_t b = grp;
    for (; b + 31u * kRedGroups < nblocks; b += 32u * kRedGroups) {
        float v[32];
#pragma unroll
        for (uint32_t j = 0; j < 32u; ++j) v[j] = partial[(size_t)(b + j * kRedGroups) * kNP + p];
#pragma unroll
        for (uint32_t j = 0; j < 32u; ++j) acc += v[j];
    }
    for (; b + 7u * kRedGroups < nblocks; b += 8u * kRedGroups) {
        float v[8];
#pragma unroll
        for (uint32_t j = 0; j < 8u; ++j) v[j] = partial[(size_t)(b + j * kRedGroups) * kNP + p];
#pragma unroll
        for (uint32_t j = 0; j < 8u; ++j) acc += v[j];
    }
    for (; b < nblocks; b += kRedGroups) acc += partial[(size_t)b * kNP + p];
    return acc;
}

// The blocks' weight sums (and, with want_loss, loss sums), by the first
// wave in a fixed order: lane l adds entries l, l + 64, l + 128, ... in
// turn, then a butterfly across the lanes gives every lane the totals.  The
// first kBlockSumPer entries of each lane are loaded by block_sums_begin,
// which the caller issues before its other loads so that the latencies
// overlap.
constexpr uint32_t kBlockSumPer = 4;

struct BlockSums {
    float w[kBlockSumPer], l[kBlockSumPer];
};

__device__ __forceinline__ void block_sums_begin(const float* part_w, const float* part_loss, uint32_t nblocks,
                                                 bool want_loss, BlockSums& b) {
#pragma unroll
    for (uint32_t k = 0; k < kBlockSumPer; ++k) {
        const uint32_t i = threadIdx.x + 64u * k;
        b.w[k] = i < nblocks ? part_w[i] : 0.0f;
        b.l[k] = want_loss && i < nblocks ? part_loss[i] : 0.0f;
    }
}

__device__ __forceinline__ void block_sums_end(const float* part_w, const float* part_loss, uint32_t nblocks,
                                               bool want_loss, const BlockSums& b, float& sw, float& sl) {
    sw = 0.0f;
    sl = 0.0f;
#pragma unroll
    for (uint32_t k = 0; k < kBlockSumPer; ++k) {
        sw += b.w[k];
        sl += b.l[k];
    }
    for (uint32_t i = threadIdx.x + 64u * kBlockSumPer; i < nblocks; i += 64u) {
        sw += part_w[i];
        if (want_loss) sl += part_loss[i];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sw += __shfl_xor(sw, off, 64);
        sl += __shfl_xor(sl, off, 64);
    }
}

// Adam on parameter p (weight w0, moments m0, v0) with gradient gr (bias
// corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t), then its BF16 operands
// refreshed.
__device__ __forceinline__ void adam_apply(uint32_t p, float gr, float w0, float m0, float v0, float* master,
                                           float* m, float* v, uint16_t* frag, float lr, float beta1, float beta2,
                                           float eps, float c1, float c2) {
    const float mm = beta1 * m0 + (1.0f - beta1) * gr;
    const float vv = beta2 * v0 + (1.0f - beta2) * (gr * gr);
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / c1, vh = vv / c2;
    const float np = w0 - lr * mh / (sqrtf(vh) + eps);
    master[p] = np;
    write_frag(frag, p, np);
}

// Sum of the blocks' partial rows, divided by the batch's sum of weights;
// then either stored (mode 0) or applied by Adam (mode 1).  A block covers
// 32 parameters with 8 row groups: group r sums rows r, r + 8, ... in order,
// and the 8 group sums are added in group order, so the result does not
// depend on scheduling.
__global__ void __launch_bounds__(kBlock) k_mlp_reduce(const float* __restrict__ partial,
                                                       const float* __restrict__ part_w,
                                                       const float* __restrict__ part_loss, uint32_t nblocks,
                                                       uint32_t mode, float* __restrict__ out,
                                                       float* __restrict__ master, float* __restrict__ m,
                                                       float* __restrict__ v, uint16_t* __restrict__ frag, float lr,
                                                       float beta1, float beta2, float eps, float c1, float c2,
                                                       float* __restrict__ loss) {
    __shared__ float s_part[kRedGroups][kRedCols];
    __shared__ float s_inv;
    const uint32_t col = threadIdx.x % kRedCols, grp = threadIdx.x / kRedCols;
    const uint32_t p = blockIdx.x * kRedCols + col;
    const bool want_loss = blockIdx.x == 0 && loss;
    const bool sums = threadIdx.x < 64u;
    BlockSums bs;
    if (sums) block_sums_begin(part_w, part_loss, nblocks, want_loss, bs);
    // the parameter's weight and moments, loaded ahead for Adam
    const bool upd = grp == 0u && p < kNP && mode != 0u;
    float w0 = 0.0f, m0 = 0.0f, v0 = 0.0f;
    if (upd) {
        w0 = master[p];
        m0 = m[p];
        v0 = v[p];
    }
    s_part[grp][col] = p < kNP ? column_sum(partial, p, grp, nblocks) : 0.0f;
    float sw = 0.0f, sl = 0.0f;
    if (sums) block_sums_end(part_w, part_loss, nblocks, want_loss, bs, sw, sl);
    if (threadIdx.x == 0) {
        const float inv = sw > 0.0f ? 1.0f / sw : 0.0f;
        s_inv = inv;
        if (want_loss) *loss = sl * inv;
    }
    __syncthreads();
    if (grp != 0 || p >= kNP) return;
    float gsum = 0.0f;
    for (uint32_t r = 0; r < kRedGroups; ++r) gsum += s_part[r][col];
    const float gr = gsum * s_inv;
    if (mode == 0u) {
        out[p] = gr;
        return;
    }
    adam_apply(p, gr, w0, m0, v0, master, m, v, frag, lr, beta1, beta2, eps, c1, c2);
}

__global__ void __launch_bounds__(kBlock) k_mlp_refresh(const float* __restrict__ master,
                                                        uint16_t* __restrict__ frag) {
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p < kNP) write_frag(frag, p, master[p]);
}

// Encoded inputs of every point, in the order the lanes of layer 1 read
// them: entry (p, kb, g) holds the 8 values of k-block kb that lane group g
// supplies for point p.
__global__ void __launch_bounds__(kBlock) k_mlp_encode(MlpEncode enc, const float* __restrict__ pos,
                                                       const float* __restrict__ nrm, uint32_t P,
                                                       bf16x8* __restrict__ out) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;  // (point, lane group)
    if (i >= 4u * P) return;
    const uint32_t p = i >> 2, g = i & 3u;
    float v[6];
    point_inputs(enc, pos, nrm, p, v);
    bf16x8 x[5];
    encode_b(v, g, x);
#pragma unroll
    for (uint32_t kb = 0; kb < 5u; ++kb) out[((size_t)p * 5u + kb) * 4u + g] = x[kb];
}

// Training order of an epoch: key of tuple i = first word of Philox at
// counter (i, epoch, 0, scene << 16 | 2); sorted (stably) by key.
__global__ void __launch_bounds__(kBlock) k_mlp_order(MlpOrder ord, uint32_t* __restrict__ out) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < ord.n) out[i] = mlp_order_at(ord, i);
}

// Initial weights: uniform in +-sqrt(6 / fan_in) (He et al. 2015, uniform
// form) from Philox at counter (p, 0, 0, scene << 16 | 3); biases zero.
__global__ void __launch_bounds__(kBlock) k_mlp_init(float* __restrict__ master, uint32_t scene_id,
                                                     uint32_t seed_lo, uint32_t seed_hi) {
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= kNP) return;
    uint32_t layer, o, j;
    if (!weight_of(p, layer, o, j)) {
        master[p] = 0.0f;
        return;
    }
    uint32_t x0 = p, x1 = 0u, x2 = 0u, x3 = (scene_id << 16) | 3u;
    philox4x32_10(x0, x1, x2, x3, seed_lo, seed_hi);
    const float a = sqrtf(6.0f / (layer == 1u ? (float)kIn : (float)kH));
    master[p] = (2.0f * unit24(x0) - 1.0f) * a;
}

inline uint32_t blocks_for(size_t n) { return (uint32_t)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_mlp_refresh(const float* master, uint16_t* frag, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_refresh, dim3(blocks_for(kNP)), dim3(kBlock), 0, s, master, frag);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const uint16_t* frag, const float* master, MlpEncode enc, const float* pos,
                              const float* nrm, uint32_t P, float* cdf, float* logits, hipStream_t s) {
    if (P == 0) return hipSuccess;
    const uint32_t groups = (P + 15u) / 16u;
    uint32_t grid = (groups + 3u) / 4u;
    if (grid > 2048u) grid = 2048u;
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(kBlock), 0, s, reinterpret_cast<const bf16x8*>(frag),
                       master, enc, pos, nrm, P, cdf, logits);
    return hipGetLastError();
}

hipError_t launch_mlp_encode(MlpEncode enc, const float* pos, const float* nrm, uint32_t P, uint16_t* out,
                             hipStream_t s) {
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_encode, dim3(blocks_for(4 * (size_t)P)), dim3(kBlock), 0, s, enc, pos, nrm, P,
                       reinterpret_cast<bf16x8*>(out));
    return hipGetLastError();
}

hipError_t launch_mlp_fwd_bwd(const uint16_t* frag, const float* master, MlpEncode enc, const float* pos,
                              const float* nrm, uint32_t P, const uint16_t* xenc, const MlpOrder& ord, uint32_t base,
                              const uint32_t* pid, const uint32_t* node, const float* w, uint32_t n, float* partial,
                              float* part_w, float* part_loss, uint32_t* err, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t grid = (n + kMlpTuplesPerBlock - 1u) / kMlpTuplesPerBlock;
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3(grid), dim3(kTrainThreads), 0, s, reinterpret_cast<const bf16x8*>(frag),
                       master, enc, pos, nrm, P, reinterpret_cast<const bf16x8*>(xenc), ord, base, pid, node, w, n,
                       partial, part_w, part_loss, err);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce(const float* partial, const float* part_w, const float* part_loss, uint32_t nblocks,
                             uint32_t mode, float* out, float* master, float* m, float* v, uint16_t* frag,
                             float lr, float beta1, float beta2, float eps, float c1, float c2, float* loss,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kNP + kRedCols - 1) / kRedCols), dim3(kBlock), 0, s, partial, part_w,
                       part_loss,
                       nblocks, mode, out, master, m, v, frag, lr, beta1, beta2, eps, c1, c2, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_order(const MlpOrder& ord, uint32_t* out, hipStream_t s) {
    if (ord.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_order, dim3(blocks_for(ord.n)), dim3(kBlock), 0, s, ord, out);
    return hipGetLastError();
}

hipError_t launch_mlp_init(float* master, uint32_t scene_id, uint32_t seed_lo, uint32_t seed_hi, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_init, dim3(blocks_for(kNP)), dim3(kBlock), 0, s, master, scene_id, seed_lo, seed_hi);
    return hipGetLastError();
}

}  // namespace rlc
