// The start-vector network: psi(bits) = W4 relu(W3 relu(W2 relu(W1 x + b1) + b2)
// + b3) + b4 with x the 32 occupation bits (16 up, 16 down) mapped to +-1,
// three hidden layers of 128.  It proposes the Lanczos start vector f_1
// (Alg. 1 asks only for a random vector of norm 1); training targets are
// ground-state amplitudes produced by the method itself.
//
// All products run on the bfloat16 matrix cores of gfx950 with float32
// accumulation (v_mfma_f32_16x16x32_bf16).  Layers are evaluated transposed,
// H_l^T = W_l H_{l-1}^T: weights are the A operand (16 output features x 32
// input features), activations the B operand (32 input features x 16
// samples), and an output tile C (16 features x 16 samples) held by a
// wavefront is exactly the B operand of the next layer once the K index is
// permuted consistently: lane group g = lane/16 owns features 4g..4g+3 of
// two adjacent 16-row tiles, so virtual k = 8g + t maps to feature
//   32 kb + (t < 4 ? 4g + t : 16 + 4g + t - 4)
// and the weights are read from LDS with the same map.  Weight gradients
// dW_l = dZ_l H_{l-1}^T are MFMA GEMMs over the sample dimension.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/ed.h"
#include "ed_common.h"
#include "ed_internal.h"
#include "ed_launch.h"

namespace ed {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// parameter layout (float32, flat): W1[128x32] b1[128] W2[128x128] b2 W3[128x128] b3 W4[1x128] b4[1]
constexpr int kIn = 32, kHid = 128;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kHid * kHid, oW4 = oB3 + kHid, oB4 = oW4 + kHid, kNParam = oB4 + 1;
static_assert(kNParam == ED_MLP_NPARAM, "parameter count");

__device__ __forceinline__ uint16_t bf16_bits(float f) {
    // round to nearest even on the top 16 bits (finite inputs)
    const uint32_t u = __builtin_bit_cast(uint32_t, f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }
// two floats rounded to bfloat16 (nearest even, as bf16_bits for finite values) in one register, lo first:
// the hardware conversion of gfx950
__device__ __forceinline__ uint32_t bf16_pack(float lo, float hi) {
    typedef float f32x2v __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2v{lo, hi}), bf16x2v));
}
// max(x, 0) in one integer max on the bits: a negative float (sign bit set) is a negative integer, a
// non-negative one keeps its bits.  fmaxf of a raw accumulator value would canonicalise it first (two
// instructions).
__device__ __forceinline__ float relu(float x) {
    return __builtin_bit_cast(float, max(__builtin_bit_cast(int, x), 0));
}
__device__ __forceinline__ __bf16 as_bf(uint16_t b) { return __builtin_bit_cast(__bf16, b); }

// LDS image of the weights (bfloat16) and biases (float32).  The weight rows
// are 256 (W2, W3) or 64 (W1) bytes long, so the 16 rows one A-operand read
// touches would all start in the same LDS bank; each row's 8-byte (W2, W3) or
// 16-byte (W1) pieces are therefore stored permuted by an XOR with the row
// (w_at, w1_at), which puts the 16 rows of a read on distinct banks.
struct MlpLds {
    uint16_t w1[kHid * kIn];      // [o][i]
    uint16_t w2[kHid * kHid];     // [o][i]   forward; transposed [i][o] in the backward kernel
    uint16_t w3[kHid * kHid];
    float b1[kHid], b2[kHid], b3[kHid], w4[kHid];   // w4 already rounded to bf16 values
    float b4;
};

// LDS index of element (row, k) of a 128-column weight matrix: 4-element piece
// k / 4 of the row XOR 2 (row % 16)
__device__ __forceinline__ int w_at(int row, int k) {
    return row * kHid + ((((k >> 2) ^ (2 * (row & 15))) << 2) | (k & 3));
}
// LDS index of element (row, k) of W1 (32 columns): 8-element piece k / 8 XOR (row / 4) % 4
__device__ __forceinline__ int w1_at(int row, int k) {
    return row * kIn + ((((k >> 3) ^ ((row >> 2) & 3)) << 3) | (k & 7));
}

__device__ void load_weights(const float *__restrict__ P, MlpLds &L, bool transpose) {
    for (int k = threadIdx.x; k < kHid * kIn; k += blockDim.x) {
        const int o = k / kIn, i = k - o * kIn;
        L.w1[w1_at(o, i)] = bf16_bits(P[oW1 + k]);
    }
    for (int k = threadIdx.x; k < kHid * kHid; k += blockDim.x) {
        const int o = k / kHid, i = k - o * kHid;
        const int dst = transpose ? w_at(i, o) : w_at(o, i);
        L.w2[dst] = bf16_bits(P[oW2 + k]);
        L.w3[dst] = bf16_bits(P[oW3 + k]);
    }
    for (int k = threadIdx.x; k < kHid; k += blockDim.x) {
        L.b1[k] = P[oB1 + k];
        L.b2[k] = P[oB2 + k];
        L.b3[k] = P[oB3 + k];
        L.w4[k] = bf16_val(bf16_bits(P[oW4 + k]));
    }
    if (threadIdx.x == 0) L.b4 = P[oB4];
    __syncthreads();
}

// A operand of a 128-wide layer: rows 16*ob + (lane % 16) of w ([row][col] with
// 128 columns, stored by w_at), virtual k block kb under the permuted map
__device__ __forceinline__ bf16x8 a_hidden(const uint16_t *w, int ob, int kb, int lane) {
    const int row = 16 * ob + (lane & 15), g = lane >> 4;
    const uint2 lo = *reinterpret_cast<const uint2 *>(w + w_at(row, 32 * kb + 4 * g));        // features 32kb+4g .. +3
    const uint2 hi = *reinterpret_cast<const uint2 *>(w + w_at(row, 32 * kb + 16 + 4 * g));   // 32kb+16+4g .. +3
    return __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
}

// A operand of layer 1 (32 inputs, natural k order; W1 stored by w1_at)
__device__ __forceinline__ bf16x8 a_first(const uint16_t *w1, int ob, int lane) {
    const int row = 16 * ob + (lane & 15), g = lane >> 4;
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(w1 + w1_at(row, 8 * g)));
}

// B operands of the next layer from eight 16x16 output tiles (bf16 bits)
__device__ __forceinline__ void tiles_to_b(const uint16_t (&h)[8][4], bf16x8 (&b)[4]) {
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int t = 0; t < 8; ++t) b[kb][t] = as_bf(t < 4 ? h[2 * kb][t] : h[2 * kb + 1][t - 4]);
}

// input feature f of sample (su, sd): bit f of su (f < 16) or bit f-16 of sd, as +-1
__device__ __forceinline__ void features_b(uint64_t su, uint64_t sd, int g, bf16x8 &b, uint16_t (&bits)[8]) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int f = 8 * g + t;
        const uint64_t w = f < 16 ? su : sd;
        const int bit = (int)((w >> (f & 15)) & 1ull);
        bits[t] = bit ? 0x3F80 : 0xBF80;   // +1 / -1 in bfloat16
        b[t] = as_bf(bits[t]);
    }
}

// one 128 -> 128 layer on a 16-sample tile: c[ob] = sum_kb A(ob,kb) B(kb)
__device__ __forceinline__ void layer_hidden(const uint16_t *w, const bf16x8 (&b)[4], f32x4 (&c)[8], int lane) {
#pragma unroll
    for (int ob = 0; ob < 8; ++ob) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hidden(w, ob, kb, lane), b[kb], acc, 0, 0, 0);
        c[ob] = acc;
    }
}

// ---------------------------------------------------------------------------
// Forward.  Sample s of the tile: (up index, down index) = idx pair, or, for the
// start vector (idx == nullptr), s = i_up * dim_dn + i_dn over all states.
// train: store X^T, H1^T, H2^T, H3^T (bf16, [feature][ld]) and out[s].
// infer: write psi[s] (float or double) into f1.
template <typename OUT, bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp_fwd(const float *__restrict__ P, const uint64_t *__restrict__ st_up,
                                                 const uint64_t *__restrict__ st_dn, const int32_t *__restrict__ idx,
                                                 int64_t n, int dim_dn, OUT *__restrict__ out, uint16_t *__restrict__ xt,
                                                 uint16_t *__restrict__ h1t, uint16_t *__restrict__ h2t,
                                                 uint16_t *__restrict__ h3t, int64_t ld) {
    __shared__ MlpLds L;
    load_weights(P, L, false);
    const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
    // training covers the padded columns up to ld too (zeros), which the
    // weight-gradient GEMMs read
    const int64_t ntile = TRAIN ? ld / 16 : (n + 15) / 16;
    const int64_t wstride = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t tile = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); tile < ntile; tile += wstride) {
        const int64_t s = tile * 16 + col;
        const bool ok = s < n;
        uint64_t su = 0, sd = 0;
        if (ok) {
            if (idx) {
                su = st_up[idx[2 * s]];
                sd = st_dn[idx[2 * s + 1]];
            } else {
                const int64_t iu = s / dim_dn;
                su = st_up[iu];
                sd = st_dn[s - iu * dim_dn];
            }
        }
        bf16x8 b1;
        uint16_t xb[8];
        features_b(su, sd, g, b1, xb);
        if (TRAIN)
#pragma unroll
            for (int t = 0; t < 8; ++t) xt[(int64_t)(8 * g + t) * ld + s] = ok ? xb[t] : (uint16_t)0;
        // layer 1
        f32x4 c[8];
#pragma unroll
        for (int ob = 0; ob < 8; ++ob) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            c[ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_first(L.w1, ob, lane), b1, acc, 0, 0, 0);
        }
        // activations as bf16 pairs: hp[ob][0] = features (4g, 4g+1), hp[ob][1] = (4g+2, 4g+3) of tile ob,
        // which is also the register layout of the next layer's B operand
        uint32_t hp[8][2];
        bf16x8 b[4];
        const float *bias[3] = {L.b1, L.b2, L.b3};
        uint16_t *store[3] = {h1t, h2t, h3t};
#pragma unroll
        for (int layer = 0; layer < 3; ++layer) {
            if (layer > 0) layer_hidden(layer == 1 ? L.w2 : L.w3, b, c, lane);
#pragma unroll
            for (int ob = 0; ob < 8; ++ob) {
                const float4 bv = *reinterpret_cast<const float4 *>(bias[layer] + 16 * ob + 4 * g);
                const float z0 = fmaxf(c[ob][0] + bv.x, 0.f), z1 = fmaxf(c[ob][1] + bv.y, 0.f);
                const float z2 = fmaxf(c[ob][2] + bv.z, 0.f), z3 = fmaxf(c[ob][3] + bv.w, 0.f);
                hp[ob][0] = bf16_pack(z0, z1);
                hp[ob][1] = bf16_pack(z2, z3);
                if (TRAIN)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int f = 16 * ob + 4 * g + i;
                        const uint16_t hb = (uint16_t)(hp[ob][i >> 1] >> (16 * (i & 1)));
                        store[layer][(int64_t)f * ld + s] = ok ? hb : (uint16_t)0;
                    }
            }
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const uint4 q = make_uint4(hp[2 * kb][0], hp[2 * kb][1], hp[2 * kb + 1][0], hp[2 * kb + 1][1]);
                b[kb] = __builtin_bit_cast(bf16x8, q);
            }
        }
        // layer 4 (128 -> 1): float32 dot of the bf16 activations with bf16 weights
        float part = 0.f;
#pragma unroll
        for (int ob = 0; ob < 8; ++ob)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t w = hp[ob][i >> 1];
                const float hv = __builtin_bit_cast(float, (i & 1) ? (w & 0xFFFF0000u) : (w << 16));
                part += hv * L.w4[16 * ob + 4 * g + i];
            }
        part += __shfl_xor(part, 16, 64);
        part += __shfl_xor(part, 32, 64);
        if (g == 0 && ok) out[s] = static_cast<OUT>(part + L.b4);
    }
}

// ---------------------------------------------------------------------------
// Inference over every state (the start vector): the forward pass of
// k_mlp_fwd with NT 16-sample tiles per wavefront, so each weight fragment
// read from LDS feeds NT matrix products instead of one.  The NT tiles are
// independent MFMA chains; the scheduling barrier after each output block
// keeps the compiler from holding every block's fragments at once.
// The accumulators start from the layer's bias (features 16 ob + 4 g .. +3 of
// this lane), so the epilogue is only the ReLU and the rounding.
template <int NT>
__device__ __forceinline__ void layer_hidden_nt(const uint16_t *w, const float *bias, const bf16x8 (&b)[NT][4],
                                                f32x4 (&c)[NT][8], int lane) {
#pragma unroll
    for (int ob = 0; ob < 8; ++ob) {
        const float4 bv = *reinterpret_cast<const float4 *>(bias + 16 * ob + 4 * (lane >> 4));
        f32x4 acc[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[q] = f32x4{bv.x, bv.y, bv.z, bv.w};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const bf16x8 a = a_hidden(w, ob, kb, lane);
#pragma unroll
            for (int q = 0; q < NT; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[q][kb], acc[q], 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < NT; ++q) c[q][ob] = acc[q];
        __builtin_amdgcn_sched_barrier(0);
    }
}

// ReLU on two bfloat16 values in one register: a negative bfloat16 is a
// negative 16-bit integer, so a packed integer max with zero clears it and keeps
// the rest (the same bits as rounding the ReLU of the float32 values).
__device__ __forceinline__ uint32_t relu_pk(uint32_t v) {
    typedef short short2v __attribute__((ext_vector_type(2)));
    const short2v r = __builtin_elementwise_max(__builtin_bit_cast(short2v, v), short2v{0, 0});
    return __builtin_bit_cast(uint32_t, r);
}

// A operand of the output layer (128 -> 1) as a 16-row product whose row 0 is
// W4 (bfloat16) and rows 1-15 are zero, under the permuted k map of a_hidden:
// row 0 of the 16x16 result is psi of the tile's 16 samples.
__device__ __forceinline__ bf16x8 a_out(const uint16_t *w4b, int kb, int lane) {
    const int g = lane >> 4;
    const uint2 lo = *reinterpret_cast<const uint2 *>(w4b + 32 * kb + 4 * g);
    const uint2 hi = *reinterpret_cast<const uint2 *>(w4b + 32 * kb + 16 + 4 * g);
    const uint32_t keep = (lane & 15) == 0 ? ~0u : 0u;
    return __builtin_bit_cast(bf16x8, make_uint4(lo.x & keep, lo.y & keep, hi.x & keep, hi.y & keep));
}

// At most 256 VGPRs (two waves per SIMD, which is also what the weights' LDS
// image allows: two workgroups per CU).
template <typename OUT, int NT>
__global__ __launch_bounds__(256, 2) void k_mlp_infer(const float *__restrict__ P, const uint64_t *__restrict__ st_up,
                                                      const uint64_t *__restrict__ st_dn, int64_t n, int dim_dn,
                                                      OUT *__restrict__ out) {
    __shared__ MlpLds L;
    __shared__ uint16_t w4b[kHid];
    load_weights(P, L, false);
    for (int k = threadIdx.x; k < kHid; k += blockDim.x) w4b[k] = bf16_bits(P[oW4 + k]);
    __syncthreads();
    const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
    const int64_t ngroup = (n + 16 * NT - 1) / (16 * NT);
    const int64_t wstride = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t grp = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); grp < ngroup; grp += wstride) {
        f32x4 c[NT][8];
        bf16x8 b[NT][4];
        // layer 1 (32 -> 128) on the occupation bits
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int64_t s = (grp * NT + q) * 16 + col;
            uint64_t su = 0, sd = 0;
            if (s < n) {
                const int64_t iu = s / dim_dn;
                su = st_up[iu];
                sd = st_dn[s - iu * dim_dn];
            }
            uint16_t xb[8];
            features_b(su, sd, g, b[q][0], xb);
        }
#pragma unroll
        for (int ob = 0; ob < 8; ++ob) {
            const bf16x8 a = a_first(L.w1, ob, lane);
            const float4 bv = *reinterpret_cast<const float4 *>(L.b1 + 16 * ob + 4 * g);
#pragma unroll
            for (int q = 0; q < NT; ++q)
                c[q][ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[q][0], f32x4{bv.x, bv.y, bv.z, bv.w}, 0, 0, 0);
        }
#pragma unroll
        for (int layer = 0; layer < 3; ++layer) {
            if (layer > 0) layer_hidden_nt<NT>(layer == 1 ? L.w2 : L.w3, layer == 1 ? L.b2 : L.b3, b, c, lane);
            // activations: bfloat16 pairs (rounded, then ReLU on the pair), which is also the register layout
            // of the next layer's B operand
#pragma unroll
            for (int q = 0; q < NT; ++q)
#pragma unroll
                for (int kb = 0; kb < 4; ++kb)
                    b[q][kb] = __builtin_bit_cast(
                        bf16x8, make_uint4(relu_pk(bf16_pack(c[q][2 * kb][0], c[q][2 * kb][1])),
                                           relu_pk(bf16_pack(c[q][2 * kb][2], c[q][2 * kb][3])),
                                           relu_pk(bf16_pack(c[q][2 * kb + 1][0], c[q][2 * kb + 1][1])),
                                           relu_pk(bf16_pack(c[q][2 * kb + 1][2], c[q][2 * kb + 1][3]))));
        }
        // layer 4 (128 -> 1) on the matrix cores: row 0 of W4 times the tile, float32 accumulation
        f32x4 o[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) o[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const bf16x8 a = a_out(w4b, kb, lane);
#pragma unroll
            for (int q = 0; q < NT; ++q) o[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[q][kb], o[q], 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int64_t s = (grp * NT + q) * 16 + col;
            if (g == 0 && s < n) out[s] = static_cast<OUT>(o[q][0] + L.b4);
        }
    }
}
constexpr int kInferTiles = 4;

// ---------------------------------------------------------------------------
// Backward chain on 16-sample tiles: g4 = 2 (out - target) / n, then
// dZ3 = (g4 w4) o [h3 > 0], dZ2 = (W3^T dZ3) o [h2 > 0], dZ1 = (W2^T dZ2) o [h1 > 0]
// (bf16 operands, float32 accumulation), stored bf16 [feature][ld]; per-workgroup
// partial sums of the bias gradients, of dW4 and db4, and of the squared error.
// partial layout per workgroup: [db1 128][db2 128][db3 128][dW4 128][db4][sse]
constexpr int kPartW = 4 * kHid + 2;

__global__ __launch_bounds__(256) void k_mlp_bwd(const float *__restrict__ P, const float *__restrict__ out,
                                                 const float *__restrict__ target, int64_t n,
                                                 const uint16_t *__restrict__ h1t, const uint16_t *__restrict__ h2t,
                                                 const uint16_t *__restrict__ h3t, uint16_t *__restrict__ dz1t,
                                                 uint16_t *__restrict__ dz2t, uint16_t *__restrict__ dz3t, int64_t ld,
                                                 float *__restrict__ partials) {
    __shared__ MlpLds L;   // w2, w3 transposed: [in][out]
    __shared__ float red[4][kPartW];
    load_weights(P, L, true);
    const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15, wv = threadIdx.x >> 6;
    // per-lane accumulators for the features this lane owns (f = 16 ob + 4 g + i)
    float db[3][8][4], dw4[8][4], db4 = 0.f, sse = 0.f;
#pragma unroll
    for (int ob = 0; ob < 8; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            db[0][ob][i] = db[1][ob][i] = db[2][ob][i] = 0.f;
            dw4[ob][i] = 0.f;
        }
    const int64_t ntile = ld / 16;   // padded columns get zero gradients
    const int64_t wstride = (int64_t)gridDim.x * (blockDim.x >> 6);
    const float inv_n = 2.0f / (float)n;
    for (int64_t tile = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv; tile < ntile; tile += wstride) {
        const int64_t s = tile * 16 + col;
        const bool ok = s < n;
        const float d = ok ? out[s] - target[s] : 0.f;
        const float g4 = inv_n * d;
        if (g == 0) { db4 += g4; sse += d * d; }
        const float g4r = bf16_val(bf16_bits(g4));
        // layer 3
        uint16_t dz[8][4];
#pragma unroll
        for (int ob = 0; ob < 8; ++ob)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int f = 16 * ob + 4 * g + i;
                const uint16_t hb = h3t[(int64_t)f * ld + s];
                const float hv = bf16_val(hb);
                const float z = hv > 0.f ? g4r * L.w4[f] : 0.f;
                db[2][ob][i] += z;
                dw4[ob][i] += g4r * hv;
                dz[ob][i] = bf16_bits(z);
                dz3t[(int64_t)f * ld + s] = dz[ob][i];
            }
        bf16x8 b[4];
        f32x4 c[8];
        const uint16_t *hprev[2] = {h2t, h1t};
        uint16_t *dzout[2] = {dz2t, dz1t};
#pragma unroll
        for (int layer = 0; layer < 2; ++layer) {
            tiles_to_b(dz, b);
            layer_hidden(layer == 0 ? L.w3 : L.w2, b, c, lane);   // W^T dZ with transposed LDS weights
#pragma unroll
            for (int ob = 0; ob < 8; ++ob)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int f = 16 * ob + 4 * g + i;
                    const float hv = bf16_val(hprev[layer][(int64_t)f * ld + s]);
                    const float z = hv > 0.f ? c[ob][i] : 0.f;
                    db[1 - layer][ob][i] += z;
                    dz[ob][i] = bf16_bits(z);
                    dzout[layer][(int64_t)f * ld + s] = dz[ob][i];
                }
        }
    }
    // reduce the per-lane sums over the 16 samples of a lane group, then over waves
#pragma unroll
    for (int ob = 0; ob < 8; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                db[0][ob][i] += __shfl_xor(db[0][ob][i], o, 64);
                db[1][ob][i] += __shfl_xor(db[1][ob][i], o, 64);
                db[2][ob][i] += __shfl_xor(db[2][ob][i], o, 64);
                dw4[ob][i] += __shfl_xor(dw4[ob][i], o, 64);
            }
    for (int o = 1; o < 64; o <<= 1) {
        db4 += __shfl_xor(db4, o, 64);
        sse += __shfl_xor(sse, o, 64);
    }
    if (col == 0) {
#pragma unroll
        for (int ob = 0; ob < 8; ++ob)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int f = 16 * ob + 4 * g + i;
                red[wv][f] = db[0][ob][i];
                red[wv][kHid + f] = db[1][ob][i];
                red[wv][2 * kHid + f] = db[2][ob][i];
                red[wv][3 * kHid + f] = dw4[ob][i];
            }
    }
    if (lane == 0) {
        red[wv][4 * kHid] = db4;
        red[wv][4 * kHid + 1] = sse;
    }
    __syncthreads();
    const int nw = blockDim.x >> 6;
    for (int k = threadIdx.x; k < kPartW; k += blockDim.x) {
        float sum = 0.f;
        for (int w = 0; w < nw; ++w) sum += red[w][k];
        partials[(int64_t)blockIdx.x * kPartW + k] = sum;
    }
}

// ---------------------------------------------------------------------------
// Weight gradients: one wavefront per 16x16 output tile, K = samples.
// dW1 = dZ1 X^T (8 x 2 tiles), dW2 = dZ2 H1^T (8 x 8), dW3 = dZ3 H2^T (8 x 8);
// extra workgroups reduce the bias / dW4 / db4 / loss partials in fixed order.
constexpr int kWTiles = 16 + 64 + 64;

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
    const uint4 q = *reinterpret_cast<const uint4 *>(p);
    bf16x8 a;
    a[0] = as_bf(q.x & 0xFFFF); a[1] = as_bf(q.x >> 16); a[2] = as_bf(q.y & 0xFFFF); a[3] = as_bf(q.y >> 16);
    a[4] = as_bf(q.z & 0xFFFF); a[5] = as_bf(q.z >> 16); a[6] = as_bf(q.w & 0xFFFF); a[7] = as_bf(q.w >> 16);
    return a;
}

__global__ __launch_bounds__(256) void k_mlp_wgrad(const uint16_t *__restrict__ xt, const uint16_t *__restrict__ h1t,
                                                   const uint16_t *__restrict__ h2t, const uint16_t *__restrict__ dz1t,
                                                   const uint16_t *__restrict__ dz2t, const uint16_t *__restrict__ dz3t,
                                                   int64_t ld, const float *__restrict__ partials, int nparts,
                                                   float *__restrict__ grad, double *__restrict__ loss, int64_t n) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
    const int tile = blockIdx.x * (blockDim.x >> 6) + wv;
    if (tile < kWTiles) {
        int layer, ob, ib;
        if (tile < 16) { layer = 0; ob = tile >> 1; ib = tile & 1; }
        else if (tile < 80) { layer = 1; ob = (tile - 16) >> 3; ib = (tile - 16) & 7; }
        else { layer = 2; ob = (tile - 80) >> 3; ib = (tile - 80) & 7; }
        const uint16_t *dz = layer == 0 ? dz1t : (layer == 1 ? dz2t : dz3t);
        const uint16_t *hp = layer == 0 ? xt : (layer == 1 ? h1t : h2t);
        const int ni = layer == 0 ? kIn : kHid;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const uint16_t *pa = dz + (int64_t)(16 * ob + col) * ld + 8 * g;
        const uint16_t *pb = hp + (int64_t)(16 * ib + col) * ld + 8 * g;
        for (int64_t s0 = 0; s0 < ld; s0 += 32)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(load8(pa + s0), load8(pb + s0), acc, 0, 0, 0);
        const int base = layer == 0 ? oW1 : (layer == 1 ? oW2 : oW3);
#pragma unroll
        for (int i = 0; i < 4; ++i) grad[base + (16 * ob + 4 * g + i) * ni + 16 * ib + col] = acc[i];
        return;
    }
    // reductions of the per-workgroup partials (fixed order)
    const int k = (tile - kWTiles) * 64 + lane;
    if (k >= kPartW) return;
    double sum = 0.0;
    for (int w = 0; w < nparts; ++w) sum += partials[(int64_t)w * kPartW + k];
    if (k < kHid) grad[oB1 + k] = (float)sum;
    else if (k < 2 * kHid) grad[oB2 + k - kHid] = (float)sum;
    else if (k < 3 * kHid) grad[oB3 + k - 2 * kHid] = (float)sum;
    else if (k < 4 * kHid) grad[oW4 + k - 3 * kHid] = (float)sum;
    else if (k == 4 * kHid) grad[oB4] = (float)sum;
    else if (loss) *loss = sum / (double)n;
}

// Adam with bias correction on the float32 master parameters.
__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ P, const float *__restrict__ G,
                                                  float *__restrict__ m, float *__restrict__ v, int n, int step,
                                                  float lr, float b1, float b2, float eps) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = G[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float mh = mk / (1.f - powf(b1, (float)step));
    const float vh = vk / (1.f - powf(b2, (float)step));
    P[k] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------
// Minibatch draws from a ground-state vector psi: with the selector u0 < 1/2
// the state is drawn with probability |psi|^2 (row by its weight, then the
// column inside the row), else uniformly; the target is sqrt(dim) psi[state].
// row_cdf: inclusive prefix sums of the row weights, normalised to 1 at the end.
template <typename T>
__global__ __launch_bounds__(256) void k_row_weights(const T *__restrict__ psi, int dim_up, int dim_dn,
                                                     double *__restrict__ w) {
    for (int r = blockIdx.x; r < dim_up; r += gridDim.x) {
        double s[1] = {0.0};
        for (int c = threadIdx.x; c < dim_dn; c += blockDim.x) {
            const double v = psi[(int64_t)r * dim_dn + c];
            s[0] += v * v;
        }
        double tot[1];
        block_sum<1>(s, tot);
        if (threadIdx.x == 0) w[r] = tot[0];
        __syncthreads();
    }
}

// inclusive prefix sums of w[0..n) in float64, normalised by the total (one
// workgroup; chunked, fixed order)
__global__ __launch_bounds__(1024) void k_cdf_scan(double *__restrict__ w, int n) {
    __shared__ double part[1024];
    const int T = blockDim.x, t = threadIdx.x;
    const int chunk = (n + T - 1) / T;
    const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
    double s = 0.0;
    for (int k = lo; k < hi; ++k) s += w[k];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        double run = 0.0;
        for (int k = 0; k < T; ++k) {
            const double v = part[k];
            part[k] = run;
            run += v;
        }
        w[n] = run;   // total, in the slot after the data
    }
    __syncthreads();
    const double total = w[n];
    double run = part[t];
    for (int k = lo; k < hi; ++k) {
        run += w[k];
        w[k] = total > 0.0 ? run / total : 0.0;
    }
}

// One wavefront per sample.  With uniforms[2k] < 1/2 the row comes from the
// row distribution (binary search of row_cdf) and the column from the row's
// own |psi|^2: the wave reads the row coalesced, once for its total and once
// in 64-element chunks with an inclusive prefix sum, and takes the first
// column whose running sum exceeds the target.  Otherwise the state is
// drawn uniformly from the position uniforms[2k+1].
constexpr int kSampleWaves = 4;   // samples per 256-thread workgroup

template <typename T>
__global__ __launch_bounds__(64 * kSampleWaves) void k_mlp_sample(const T *__restrict__ psi, int dim_up, int dim_dn,
                                                                  const double *__restrict__ row_cdf,
                                                                  const double *__restrict__ uni, int n,
                                                                  int32_t *__restrict__ idx,
                                                                  float *__restrict__ target) {
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * kSampleWaves + (threadIdx.x >> 6);
    if (k >= n) return;   // the whole wave
    const double sel = uni[2 * k], u = uni[2 * k + 1];
    int r, c;
    if (sel < 0.5) {
        int lo = 0, hi = dim_up - 1;   // first row with cdf > u
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (row_cdf[mid] > u) hi = mid; else lo = mid + 1;
        }
        r = lo;
        const double prev = r > 0 ? row_cdf[r - 1] : 0.0;
        const double width = row_cdf[r] - prev;
        const double rem = width > 0.0 ? (u - prev) / width : 0.0;   // position inside the row, in [0, 1)
        const T *row = psi + (int64_t)r * dim_dn;
        double tot = 0.0;
        for (int cc = lane; cc < dim_dn; cc += 64) {
            const double v = row[cc];
            tot += v * v;
        }
        for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
        const double want = rem * tot;
        double acc = 0.0;   // sum of the chunks before this one
        c = dim_dn - 1;
        for (int base = 0; base < dim_dn; base += 64) {
            const int cc = base + lane;
            double pre = 0.0;
            if (cc < dim_dn) {
                const double v = row[cc];
                pre = v * v;
            }
            for (int o = 1; o < 64; o <<= 1) {
                const double y = __shfl_up(pre, o, 64);
                if (lane >= o) pre += y;
            }
            const unsigned long long hit = __ballot(cc < dim_dn && acc + pre > want);
            if (hit) {
                c = base + __ffsll((long long)hit) - 1;
                break;
            }
            acc += __shfl(pre, 63, 64);
        }
    } else {
        const int64_t s = min((int64_t)(u * (double)dim_up * (double)dim_dn), (int64_t)dim_up * dim_dn - 1);
        r = (int)(s / dim_dn);
        c = (int)(s - (int64_t)r * dim_dn);
    }
    if (lane == 0) {
        idx[2 * k] = r;
        idx[2 * k + 1] = c;
        target[k] = (float)(sqrt((double)dim_up * (double)dim_dn) * (double)psi[(int64_t)r * dim_dn + c]);
    }
}

// workspace layout for a minibatch of n samples (ld = n rounded up to 32)
struct MlpWs {
    uint16_t *xt, *h1t, *h2t, *h3t, *dz1t, *dz2t, *dz3t;
    float *out, *parts;
    int64_t ld;
    int nparts;
};
constexpr int kBwdBlocks = 64;

static int64_t mlp_ld(int64_t n) { return (n + 31) / 32 * 32; }

static int64_t mlp_ws_bytes(int64_t n) {
    const int64_t ld = mlp_ld(n);
    auto al = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    return al(2 * kIn * ld) + 6 * al(2 * kHid * ld) + al(4 * ld) + al(4 * (int64_t)kBwdBlocks * kPartW);
}

static MlpWs mlp_ws(void *ws, int64_t n) {
    auto al = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    MlpWs w;
    w.ld = mlp_ld(n);
    char *p = static_cast<char *>(ws);
    w.xt = reinterpret_cast<uint16_t *>(p); p += al(2 * kIn * w.ld);
    uint16_t **hs[6] = {&w.h1t, &w.h2t, &w.h3t, &w.dz1t, &w.dz2t, &w.dz3t};
    for (auto hp : hs) { *hp = reinterpret_cast<uint16_t *>(p); p += al(2 * kHid * w.ld); }
    w.out = reinterpret_cast<float *>(p); p += al(4 * w.ld);
    w.parts = reinterpret_cast<float *>(p);
    w.nparts = kBwdBlocks;
    return w;
}

static int fwd_grid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 63) / 64, 4096)); }

}  // namespace ed

using namespace ed;

extern "C" {

int ed_mlp_workspace_size(int64_t n, int64_t *bytes) {
    clear_error();
    if (n < 1 || n > (1 << 24) || !bytes) return set_error(ED_EINVAL, "ed_mlp_workspace_size: bad arguments");
    *bytes = mlp_ws_bytes(n);
    return ED_OK;
}

int ed_mlp_forward(const float *params, const uint64_t *st_up, const uint64_t *st_dn, const int32_t *idx, int64_t n,
                   float *out, void *ws, void *stream) {
    clear_error();
    if (!params || !st_up || !st_dn || !idx || n < 1 || n > (1 << 24) || !ws)
        return set_error(ED_EINVAL, "ed_mlp_forward: bad arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const MlpWs w = mlp_ws(ws, n);
    float *o = out ? out : w.out;
    hipLaunchKernelGGL((k_mlp_fwd<float, true>), dim3(fwd_grid(n)), dim3(256), 0, s, params, st_up, st_dn, idx, n, 0,
                       o, w.xt, w.h1t, w.h2t, w.h3t, w.ld);
    ED_LAUNCHED("k_mlp_fwd");
    if (out && out != w.out) ED_HIP(hipMemcpyAsync(w.out, out, 4 * (size_t)n, hipMemcpyDeviceToDevice, s));
    return ED_OK;
}

int ed_mlp_backward(const float *params, const float *target, int64_t n, float *grad, double *loss, void *ws,
                    void *stream) {
    clear_error();
    if (!params || !target || n < 1 || n > (1 << 24) || !grad || !ws)
        return set_error(ED_EINVAL, "ed_mlp_backward: bad arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const MlpWs w = mlp_ws(ws, n);
    hipLaunchKernelGGL(k_mlp_bwd, dim3(w.nparts), dim3(256), 0, s, params, w.out, target, n, w.h1t, w.h2t, w.h3t,
                       w.dz1t, w.dz2t, w.dz3t, w.ld, w.parts);
    ED_LAUNCHED("k_mlp_bwd");
    const int red_waves = (kPartW + 63) / 64;
    const int waves = kWTiles + red_waves;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((waves + 3) / 4), dim3(256), 0, s, w.xt, w.h1t, w.h2t, w.dz1t, w.dz2t,
                       w.dz3t, w.ld, w.parts, w.nparts, grad, loss, n);
    ED_LAUNCHED("k_mlp_wgrad");
    return ED_OK;
}

int ed_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t step, float lr, float beta1,
                float beta2, float eps, void *stream) {
    clear_error();
    if (!params || !grad || !m || !v || step < 1) return set_error(ED_EINVAL, "ed_mlp_adam: bad arguments");
    hipLaunchKernelGGL(k_mlp_adam, dim3((kNParam + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                       params, grad, m, v, kNParam, step, lr, beta1, beta2, eps);
    ED_LAUNCHED("k_mlp_adam");
    return ED_OK;
}

int ed_mlp_start_vector(const float *params, const ed_ham *h, void *f1, void *stream) {
    clear_error();
    int rc = check_real(h, "ed_mlp_start_vector");
    if (rc) return rc;
    if (!params || !f1) return set_error(ED_EINVAL, "ed_mlp_start_vector: bad arguments");
    const int64_t n = h->dim_up * h->dim_dn;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (h->dtype == ED_F64)
        hipLaunchKernelGGL((k_mlp_infer<double, kInferTiles>), dim3(fwd_grid(n)), dim3(256), 0, s, params, h->st_up,
                           h->st_dn, n, (int)h->dim_dn, (double *)f1);
    else
        hipLaunchKernelGGL((k_mlp_infer<float, kInferTiles>), dim3(fwd_grid(n)), dim3(256), 0, s, params, h->st_up,
                           h->st_dn, n, (int)h->dim_dn, (float *)f1);
    ED_LAUNCHED("k_mlp_infer");
    return ED_OK;
}

int ed_mlp_row_cdf(const void *psi, const ed_ham *h, double *cdf, void *stream) {
    clear_error();
    int rc = check_real(h, "ed_mlp_row_cdf");
    if (rc) return rc;
    if (!psi || !cdf) return set_error(ED_EINVAL, "ed_mlp_row_cdf: bad arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int grid = (int)std::min<int64_t>(h->dim_up, 4096);
    if (h->dtype == ED_F64)
        hipLaunchKernelGGL(k_row_weights<double>, dim3(grid), dim3(256), 0, s, (const double *)psi, (int)h->dim_up,
                           (int)h->dim_dn, cdf);
    else
        hipLaunchKernelGGL(k_row_weights<float>, dim3(grid), dim3(256), 0, s, (const float *)psi, (int)h->dim_up,
                           (int)h->dim_dn, cdf);
    ED_LAUNCHED("k_row_weights");
    hipLaunchKernelGGL(k_cdf_scan, dim3(1), dim3(1024), 0, s, cdf, (int)h->dim_up);
    ED_LAUNCHED("k_cdf_scan");
    return ED_OK;
}

int ed_mlp_sample(const void *psi, const ed_ham *h, const double *row_cdf, const double *uniforms, int32_t n,
                  int32_t *idx, float *target, void *stream) {
    clear_error();
    int rc = check_real(h, "ed_mlp_sample");
    if (rc) return rc;
    if (!psi || !row_cdf || !uniforms || n < 1 || !idx || !target)
        return set_error(ED_EINVAL, "ed_mlp_sample: bad arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int grid = (n + kSampleWaves - 1) / kSampleWaves;
    if (h->dtype == ED_F64)
        hipLaunchKernelGGL(k_mlp_sample<double>, dim3(grid), dim3(64 * kSampleWaves), 0, s, (const double *)psi, (int)h->dim_up,
                           (int)h->dim_dn, row_cdf, uniforms, n, idx, target);
    else
        hipLaunchKernelGGL(k_mlp_sample<float>, dim3(grid), dim3(64 * kSampleWaves), 0, s, (const float *)psi, (int)h->dim_up,
                           (int)h->dim_dn, row_cdf, uniforms, n, idx, target);
    ED_LAUNCHED("k_mlp_sample");
    return ED_OK;
}

}  // extern "C"
