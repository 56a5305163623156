// Internal interface of the learned proposal's kernels (mlp.hip): sizes,
// the input encoding's parameters, the epoch order and the launches.
#pragma once

#include "rlc_internal.h"

namespace rlc {

// mlp.hip: the learned proposal (144 -> 64 -> 64 -> 64 -> 64, BF16 MFMA)
constexpr uint32_t kMlpParams = 64u * 144u + 64u + 3u * (64u * 64u + 64u);
constexpr uint32_t kMlpFragVecs = 4352u;   // 16-byte BF16 operand fragments
constexpr uint32_t kMlpTuplesPerBlock = 128u;  // training tuples per block of the fused kernel
struct MlpEncode {
    float lo[3];
    float ext[3];
};

// The order in which an epoch visits the training tuples (the paper leaves
// it open): position i holds tuple pi(i), pi a keyed permutation of 0..n-1
// computed per position, so no sort is needed.  pi is an eight-round
// balanced Feistel network on 2h-bit words, 4^h >= n (Luby and Rackoff),
// whose round r maps halves (L, R) to (R, L xor (fmix32(R xor k_r) mod
// 2^h)) with MurmurHash3's finaliser; values of n or more go through the
// network again until one is below n (cycle walking, Black and Rogaway).
// The round keys are the words of Philox at counters (j, epoch, 0,
// scene << 16 | 2), j = 0, 1.  n == 0 stands for the identity.
struct MlpOrder {
    uint32_t n;
    uint32_t h;
    uint32_t k[8];
};

__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t v) {
    v ^= v >> 16;
    v *= 0x85EBCA6Bu;
    v ^= v >> 13;
    v *= 0xC2B2AE35u;
    v ^= v >> 16;
    return v;
}

__host__ __device__ __forceinline__ uint32_t mlp_order_at(const MlpOrder& o, uint32_t i) {
    if (o.n == 0u) return i;  // the identity
    const uint32_t h = o.h, mask = (uint32_t)((1ull << h) - 1ull);
    uint32_t x = i;
    do {
        uint32_t hi = (uint32_t)((unsigned long long)x >> h), lo = x & mask;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint32_t t = hi ^ (fmix32(lo ^ o.k[r]) & mask);
            hi = lo;
            lo = t;
        }
        x = (uint32_t)(((unsigned long long)hi << h) | lo);
    } while (x >= o.n);  // a permutation of 0..4^h-1: the walk returns below n
    return x;
}

inline MlpOrder mlp_epoch_order(uint32_t n, uint32_t epoch, uint32_t scene_id, unsigned long long seed) {
    MlpOrder o{};
    o.n = n;
    o.h = 1;
    while ((1ull << (2u * o.h)) < (unsigned long long)n) ++o.h;
    for (uint32_t j = 0; j < 2u; ++j) {
        uint32_t x0 = j, x1 = epoch, x2 = 0u, x3 = (scene_id << 16) | 2u;
        philox4x32_10(x0, x1, x2, x3, (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32));
        o.k[4 * j] = x0;
        o.k[4 * j + 1] = x1;
        o.k[4 * j + 2] = x2;
        o.k[4 * j + 3] = x3;
    }
    return o;
}
hipError_t launch_mlp_refresh(const float* master, uint16_t* frag, hipStream_t s);
hipError_t launch_mlp_forward(const uint16_t* frag, const float* master, MlpEncode enc, const float* pos,
                              const float* nrm, uint32_t P, float* cdf, float* logits, hipStream_t s);
// Encoded inputs of P points for the training kernel: kMlpEncodeHalves
// BF16 values (320 bytes) per point.
constexpr uint32_t kMlpEncodeHalves = 160u;
hipError_t launch_mlp_encode(MlpEncode enc, const float* pos, const float* nrm, uint32_t P, uint16_t* out,
                             hipStream_t s);
// xenc: the points' encoded inputs (launch_mlp_encode), or null to encode
// in the kernel.  The n tuples are those at positions base .. base + n - 1
// of the order ord.
hipError_t launch_mlp_fwd_bwd(const uint16_t* frag, const float* master, MlpEncode enc, const float* pos,
                              const float* nrm, uint32_t P, const uint16_t* xenc, const MlpOrder& ord, uint32_t base,
                              const uint32_t* pid, const uint32_t* node, const float* w, uint32_t n, float* partial,
                              float* part_w, float* part_loss, uint32_t* err, hipStream_t s);
hipError_t launch_mlp_order(const MlpOrder& ord, uint32_t* out, hipStream_t s);
// mode 0: write the batch gradient to `out`; mode 1: Adam step on master
// (m, v), then refresh the BF16 fragments
hipError_t launch_mlp_reduce(const float* partial, const float* part_w, const float* part_loss, uint32_t nblocks,
                             uint32_t mode, float* out, float* master, float* m, float* v, uint16_t* frag,
                             float lr, float beta1, float beta2, float eps, float c1, float c2, float* loss,
                             hipStream_t s);
hipError_t launch_mlp_init(float* master, uint32_t scene_id, uint32_t seed_lo, uint32_t seed_hi, hipStream_t s);

}  // namespace rlc
