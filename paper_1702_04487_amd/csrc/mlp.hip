// mlp.hip -- the surrogate network of the droplet outputs: a multilayer
// perceptron 7 -> 128 -> 128 -> 4 with GELU, trained and evaluated with
// bfloat16 matrix-core (MFMA) products and float32 accumulation, float32
// master weights and Adam, for an ensemble of members.
//
// Inputs: contact angle, surface tension, the two pulse amplitudes and the
// three durations of Fig. 1; outputs: breakup step, drop velocity, drop
// volume (regression, normalised) and the satellite flag (logit).
//
// Padded layouts (per member, row-major):
//   W1 [128][16]  (inputs 7..15 zero)   b1 [128]
//   W2 [128][128]                         b2 [128]
//   W3 [16][128]  (outputs 4..15 zero)   b3 [16]
// Matrix-core products: v_mfma_f32_16x16x32_bf16 (gfx950), D[16x16] +=
// A[16x32] B[32x16], with lane l holding A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16] for j = 0..7; where the inner dimension leaves 16
// (the first layer's 16 padded inputs, minibatches of an odd number of 16-row
// tiles) v_mfma_f32_16x16x16_bf16, with A[l % 16][4 (l / 16) + q] and
// B[4 (l / 16) + q][l % 16].  Both give D[4 (l / 16) + q][l % 16], q = 0..3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "mlp_core.h"

namespace ij {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int MT = 256;         // threads of the inference and refresh workgroups
constexpr int MT_TRAIN = 1024;  // threads of the training workgroup

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16) | ((u & 0xffffu) ? 0x40 : 0);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// acc += A[r0 .. r0+15][0..K) B[0..K)[c0 .. c0+15] on one wave; element (r, k)
// of A is A[r * ars + k * acs], element (k, c) of B is B[k * brs + c * bcs].
__device__ __forceinline__ f32x4 mma16(const uint16_t* A, int ars, int acs, const uint16_t* B, int brs, int bcs,
                                       int r0, int c0, int K, f32x4 acc)
{
    const int lane = threadIdx.x & 63;
    const int i = lane & 15;
    int k0 = 0;
    for (const int k8 = 8 * (lane >> 4); k0 + 32 <= K; k0 += 32) {
        bf16x8 a, b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            a[j] = __builtin_bit_cast(__bf16, A[(size_t)(r0 + i) * ars + (size_t)(k0 + k8 + j) * acs]);
            b[j] = __builtin_bit_cast(__bf16, B[(size_t)(k0 + k8 + j) * brs + (size_t)(c0 + i) * bcs]);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    if (k0 < K) {   // the last 16 of the inner dimension
        const int kq = 4 * (lane >> 4);
        bf16x4 a, b;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[q] = (short)A[(size_t)(r0 + i) * ars + (size_t)(k0 + kq + q) * acs];
            b[q] = (short)B[(size_t)(k0 + kq + q) * brs + (size_t)(c0 + i) * bcs];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// row and column of element q of the tile a lane holds
__device__ __forceinline__ int tile_row(int q) { return 4 * ((threadIdx.x & 63) >> 4) + q; }
__device__ __forceinline__ int tile_col() { return threadIdx.x & 15; }

struct Member {
    float* w;          // master float32 parameters (padded layout)
    float* m;          // Adam first moments
    float* v;          // Adam second moments
    float* g;          // gradients
    uint16_t* wb;      // bfloat16 copies of W1, W2, W3
};

__device__ __forceinline__ Member member(const MlpDev& D, int k)
{
    Member r;
    r.w = D.w + (size_t)k * kMlpParams;
    r.m = D.m + (size_t)k * kMlpParams;
    r.v = D.v + (size_t)k * kMlpParams;
    r.g = D.g + (size_t)k * kMlpParams;
    r.wb = D.wb + (size_t)k * kMlpWeightsBf16;
    return r;
}

// Forward pass of S16 rows (a multiple of 16) whose normalised inputs are
// in xn [S16][16]; z1, z2 float32 and a1, a2 bfloat16 [S16][128].  The
// third layer's 16 x 16 output tiles go to `epilogue(row tile, acc)`.
template <typename Epi>
__device__ void forward_rows(const Member& P, const uint16_t* xn, float* z1, uint16_t* a1, float* z2, uint16_t* a2,
                             int S16, Epi epilogue)
{
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int T = S16 / 16;
    const uint16_t* W1b = P.wb + kMlpW1b;
    const uint16_t* W2b = P.wb + kMlpW2b;
    const uint16_t* W3b = P.wb + kMlpW3b;
    // layer 1: z1 = xn W1^T + b1 (B[k][c] = W1[c][k])
    for (int it = wave; it < T * 8; it += nw) {
        const int rt = it >> 3, nt = it & 7;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma16(xn, 16, 1, W1b, 1, 16, rt * 16, nt * 16, 16, acc);
        const int c = nt * 16 + tile_col();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = rt * 16 + tile_row(q);
            const float z = acc[q] + P.w[kMlpB1 + c];
            z1[(size_t)r * 128 + c] = z;
            a1[(size_t)r * 128 + c] = to_bf16(gelu(z));
        }
    }
    __syncthreads();
    // layer 2: z2 = a1 W2^T + b2
    for (int it = wave; it < T * 8; it += nw) {
        const int rt = it >> 3, nt = it & 7;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma16(a1, 128, 1, W2b, 1, 128, rt * 16, nt * 16, 128, acc);
        const int c = nt * 16 + tile_col();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = rt * 16 + tile_row(q);
            const float z = acc[q] + P.w[kMlpB2 + c];
            z2[(size_t)r * 128 + c] = z;
            a2[(size_t)r * 128 + c] = to_bf16(gelu(z));
        }
    }
    __syncthreads();
    // layer 3: o = a2 W3^T + b3 (16 padded outputs)
    for (int rt = wave; rt < T; rt += nw) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma16(a2, 128, 1, W3b, 1, 128, rt * 16, 0, 128, acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += P.w[kMlpB3 + tile_col()];
        epilogue(rt, acc);
    }
    __syncthreads();
}

}  // namespace

// bfloat16 copies of the three weight matrices of one member
__device__ void mlp_refresh_bf16(const float* w, uint16_t* wb, int t, int nt)
{
    for (int k = t; k < kMlpW1Size; k += nt) wb[kMlpW1b + k] = to_bf16(w[kMlpW1 + k]);
    for (int k = t; k < kMlpW2Size; k += nt) wb[kMlpW2b + k] = to_bf16(w[kMlpW2 + k]);
    for (int k = t; k < kMlpW3Size; k += nt) wb[kMlpW3b + k] = to_bf16(w[kMlpW3 + k]);
}

// ----------------------------------------------------------------- training
//
// One workgroup of MT_TRAIN threads (16 waves: the phases below are split
// over waves, and more waves hide the latency of each wave's chain of
// matrix-core products) per ensemble member runs one minibatch step: the rows are
// idx[member][step][0..S) of (X, Y), or rows 0..S-1 when idx is null.
// mode 0: gradients into P.g and an Adam update (step number adam_t);
// mode 1: gradients only.  loss_out[member] (if set) gets the minibatch loss.
__global__ __launch_bounds__(MT_TRAIN) void k_mlp_step(MlpDev D, MlpNorm N, const float* __restrict__ X,
                                                 const float* __restrict__ Y, int n_rows, const int* __restrict__ idx,
                                                 int step, int steps, int S, float lr, int adam_t, int mode,
                                                 float* __restrict__ loss_out)
{
    const int mem = blockIdx.x;
    const Member P = member(D, mem);
    const int S16 = (S + 15) & ~15;
    // per-member scratch
    MlpScratch W = mlp_scratch(D, mem);
    const int t = threadIdx.x;
    __shared__ float s_loss;
    __shared__ int s_rows[kMlpMaxBatch];
    if (t == 0) s_loss = 0.f;
    for (int r = t; r < S16; r += MT_TRAIN) {
        int src = -1;
        if (r < S) src = idx ? min(max(idx[((size_t)mem * steps + step) * S + r], 0), n_rows - 1) : r;
        s_rows[r] = src;
    }
    __syncthreads();
    // normalised inputs, padded rows and columns zero
    for (int e = t; e < S16 * 16; e += MT_TRAIN) {
        const int r = e >> 4, c = e & 15;
        const int src = s_rows[r];
        float v = 0.f;
        if (src >= 0 && c < kMlpIn) v = (X[(size_t)src * kMlpIn + c] - N.x_mean[c]) * N.x_inv_std[c];
        W.xn[e] = to_bf16(v);
    }
    __syncthreads();
    const float inv_s = 1.0f / (float)S;
    forward_rows(P, W.xn, W.z1, W.a1, W.z2, W.a2, S16, [&](int rt, f32x4 acc) {
        // loss gradient of the outputs: regression (2/3)(o - t)/S on
        // normalised targets, logistic (sigmoid(o) - y)/S on the flag
        const int c = tile_col();
        float lsum = 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = rt * 16 + tile_row(q);
            const int src = s_rows[r];
            float d = 0.f;
            if (src >= 0 && c < kMlpOut) {
                const float o = acc[q];
                const float y = Y[(size_t)src * kMlpOut + c];
                if (c < kMlpReg) {
                    const float tn = (y - N.y_mean[c]) * N.y_inv_std[c];
                    d = 2.0f / (float)kMlpReg * (o - tn) * inv_s;
                    lsum += (o - tn) * (o - tn) / (float)kMlpReg * inv_s;
                } else {
                    const float sg = 1.0f / (1.0f + expf(-o));
                    d = (sg - y) * inv_s;
                    lsum += (fmaxf(o, 0.f) + log1pf(expf(-fabsf(o))) - y * o) * inv_s;
                }
            }
            W.dof[(size_t)r * 16 + c] = d;
            W.dob[(size_t)r * 16 + c] = to_bf16(d);
        }
        atomicAdd(&s_loss, lsum);
    });
    // dZ2 = (dO W3) * gelu'(z2)     (B[k][c] = W3[k][c])
    const int wave = t >> 6;
    const int T = S16 / 16;
    for (int it = wave; it < T * 8; it += MT_TRAIN / 64) {
        const int rt = it >> 3, nt = it & 7;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma16(W.dob, 16, 1, P.wb + kMlpW3b, 128, 1, rt * 16, nt * 16, 16, acc);
        const int c = nt * 16 + tile_col();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const size_t k = (size_t)(rt * 16 + tile_row(q)) * 128 + c;
            const float d = acc[q] * gelu_grad(W.z2[k]);
            W.dzf[k] = d;
            W.dzb[k] = to_bf16(d);
        }
    }
    __syncthreads();
    // dW3 = dO^T a2 [16][128]; db3 = sum dO
    for (int it = wave; it < 8; it += MT_TRAIN / 64) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma16(W.dob, 1, 16, W.a2, 128, 1, 0, it * 16, S16, acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) P.g[kMlpW3 + tile_row(q) * 128 + it * 16 + tile_col()] = acc[q];
    }
    if (t < 16) {
        float s = 0.f;
        for (int r = 0; r < S16; ++r) s += W.dof[(size_t)r * 16 + t];
        P.g[kMlpB3 + t] = s;
    }
    // dW2 = dZ2^T a1 [128][128]; db2 = sum dZ2
    for (int it = wave; it < 64; it += MT_TRAIN / 64) {
        const int rt = it >> 3, nt = it & 7;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma16(W.dzb, 1, 128, W.a1, 128, 1, rt * 16, nt * 16, S16, acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) P.g[kMlpW2 + (rt * 16 + tile_row(q)) * 128 + nt * 16 + tile_col()] = acc[q];
    }
    if (t < 128) {
        float s = 0.f;
        for (int r = 0; r < S16; ++r) s += W.dzf[(size_t)r * 128 + t];
        P.g[kMlpB2 + t] = s;
    }
    __syncthreads();
    // dZ1 = (dZ2 W2) * gelu'(z1)     (B[k][c] = W2[k][c])
    for (int it = wave; it < T * 8; it += MT_TRAIN / 64) {
        const int rt = it >> 3, nt = it & 7;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma16(W.dzb, 128, 1, P.wb + kMlpW2b, 128, 1, rt * 16, nt * 16, 128, acc);
        const int c = nt * 16 + tile_col();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const size_t k = (size_t)(rt * 16 + tile_row(q)) * 128 + c;
            const float d = acc[q] * gelu_grad(W.z1[k]);
            W.dz1f[k] = d;
            W.dz1b[k] = to_bf16(d);
        }
    }
    __syncthreads();
    // dW1 = dZ1^T xn [128][16] (columns >= 7 zero); db1 = sum dZ1
    for (int it = wave; it < 8; it += MT_TRAIN / 64) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma16(W.dz1b, 1, 128, W.xn, 16, 1, it * 16, 0, S16, acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = tile_col();
            P.g[kMlpW1 + (it * 16 + tile_row(q)) * 16 + c] = c < kMlpIn ? acc[q] : 0.f;
        }
    }
    if (t < 128) {
        float s = 0.f;
        for (int r = 0; r < S16; ++r) s += W.dz1f[(size_t)r * 128 + t];
        P.g[kMlpB1 + t] = s;
    }
    __syncthreads();
    if (t == 0 && loss_out) loss_out[(size_t)mem * steps + step] = s_loss;
    if (mode != 0) return;
    // Adam (float32 masters; padding keeps zero gradients and stays zero)
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = (float)(1.0 / (1.0 - pow(0.9, (double)adam_t)));
    const float c2 = (float)(1.0 / (1.0 - pow(0.999, (double)adam_t)));
    for (int k = t; k < kMlpParams; k += MT_TRAIN) {
        const float g = P.g[k];
        const float m = b1 * P.m[k] + (1.0f - b1) * g;
        const float v = b2 * P.v[k] + (1.0f - b2) * g * g;
        P.m[k] = m;
        P.v[k] = v;
        P.w[k] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
    }
    __syncthreads();
    mlp_refresh_bf16(P.w, P.wb, t, MT_TRAIN);
}

__global__ void k_mlp_refresh(MlpDev D)
{
    const Member P = member(D, blockIdx.x);
    mlp_refresh_bf16(P.w, P.wb, threadIdx.x, blockDim.x);
}

// ---------------------------------------------------------------- inference
//
// four (eight) consecutive bfloat16 values, 8-byte (16-byte) aligned, as one
// fragment of the 16x16x16 (16x16x32) product
__device__ __forceinline__ bf16x4 frag4(const uint16_t* p) { return *reinterpret_cast<const bf16x4*>(p); }
__device__ __forceinline__ bf16x8 frag8(const uint16_t* p) { return *reinterpret_cast<const bf16x8*>(p); }

// grid (query blocks of kInferRows * MT / 64, member): each wave evaluates
// kInferRows queries (two row tiles) through the three layers with bfloat16
// products staged in LDS.  Every operand fragment is four consecutive k
// values (a 64-bit load), and each weight fragment feeds both row tiles.
// out[member][q][0..3] holds the regression outputs in target units and the
// satellite probability.
constexpr int kInferRows = 32;
constexpr int kInferTiles = kInferRows / 16;

__global__ __launch_bounds__(MT) void k_mlp_infer(MlpDev D, MlpNorm N, const float* __restrict__ X, int n,
                                                  float* __restrict__ out)
{
    const int mem = blockIdx.y;
    const Member P = member(D, mem);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 15, kq = 4 * (lane >> 4), k8 = 8 * (lane >> 4);
    const int q0 = (blockIdx.x * (MT / 64) + wave) * kInferRows;
    __shared__ __align__(16) uint16_t s_x[MT / 64][kInferRows * 16];
    __shared__ __align__(16) uint16_t s_a[MT / 64][2][kInferRows * 128];
    uint16_t* xn = s_x[wave];
    uint16_t* a1 = s_a[wave][0];
    uint16_t* a2 = s_a[wave][1];
    for (int e = lane; e < kInferRows * 16; e += 64) {
        const int r = e >> 4, c = e & 15;
        float v = 0.f;
        if (q0 + r < n && c < kMlpIn) v = (X[(size_t)(q0 + r) * kMlpIn + c] - N.x_mean[c]) * N.x_inv_std[c];
        xn[e] = to_bf16(v);
    }
    __syncthreads();
    // layer 1 (K = 16) and layer 2 (K = 128): column tile by column tile
    const uint16_t* W1 = P.wb + kMlpW1b;
    const uint16_t* W2 = P.wb + kMlpW2b;
    const uint16_t* W3 = P.wb + kMlpW3b;
    for (int nt = 0; nt < 8; ++nt) {
        const bf16x4 b = frag4(W1 + (nt * 16 + i) * 16 + kq);
        const int c = nt * 16 + tile_col();
        const float bias = P.w[kMlpB1 + c];
#pragma unroll
        for (int rt = 0; rt < kInferTiles; ++rt) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(frag4(xn + (rt * 16 + i) * 16 + kq), b, acc, 0, 0, 0);
#pragma unroll
            for (int q = 0; q < 4; ++q) a1[(rt * 16 + tile_row(q)) * 128 + c] = to_bf16(gelu(acc[q] + bias));
        }
    }
    __syncthreads();
    for (int nt = 0; nt < 8; ++nt) {
        f32x4 acc[kInferTiles];
#pragma unroll
        for (int rt = 0; rt < kInferTiles; ++rt) acc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < 128; k0 += 32) {
            const bf16x8 b = frag8(W2 + (nt * 16 + i) * 128 + k0 + k8);
#pragma unroll
            for (int rt = 0; rt < kInferTiles; ++rt)
                acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag8(a1 + (rt * 16 + i) * 128 + k0 + k8), b,
                                                                 acc[rt], 0, 0, 0);
        }
        const int c = nt * 16 + tile_col();
        const float bias = P.w[kMlpB2 + c];
#pragma unroll
        for (int rt = 0; rt < kInferTiles; ++rt)
#pragma unroll
            for (int q = 0; q < 4; ++q) a2[(rt * 16 + tile_row(q)) * 128 + c] = to_bf16(gelu(acc[rt][q] + bias));
    }
    __syncthreads();
    // layer 3: one column tile (the four outputs and padding)
    f32x4 acc[kInferTiles];
#pragma unroll
    for (int rt = 0; rt < kInferTiles; ++rt) acc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < 128; k0 += 32) {
        const bf16x8 b = frag8(W3 + i * 128 + k0 + k8);
#pragma unroll
        for (int rt = 0; rt < kInferTiles; ++rt)
            acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag8(a2 + (rt * 16 + i) * 128 + k0 + k8), b, acc[rt],
                                                             0, 0, 0);
    }
    const int c = tile_col();
    if (c < kMlpOut) {
        const float bias = P.w[kMlpB3 + c];
#pragma unroll
        for (int rt = 0; rt < kInferTiles; ++rt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = q0 + rt * 16 + tile_row(q);
                if (r >= n) continue;
                const float o = acc[rt][q] + bias;
                out[((size_t)mem * n + r) * kMlpOut + c] =
                    c < kMlpReg ? o * N.y_std[c] + N.y_mean[c] : 1.0f / (1.0f + expf(-o));
            }
    }
}

// mean and spread (population standard deviation) over the members
__global__ void k_mlp_reduce(const float* __restrict__ members, int n_members, int n, float* __restrict__ mean,
                             float* __restrict__ spread)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * kMlpOut) return;
    float s = 0.f;
    for (int k = 0; k < n_members; ++k) s += members[(size_t)k * n * kMlpOut + e];
    const float mu = s / (float)n_members;
    float v = 0.f;
    for (int k = 0; k < n_members; ++k) {
        const float d = members[(size_t)k * n * kMlpOut + e] - mu;
        v += d * d;
    }
    mean[e] = mu;
    spread[e] = sqrtf(v / (float)n_members);
}

// ---------------------------------------------------------------- launchers

hipError_t mlp_launch_step(const MlpDev& D, const MlpNorm& N, const float* X, const float* Y, int n_rows,
                           const int* idx, int step, int steps, int S, float lr, int adam_t, int mode,
                           float* loss_out, hipStream_t st)
{
    if (S < 1 || S > kMlpMaxBatch || n_rows < 1 || (!idx && S > n_rows)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_step, dim3(D.n_members), dim3(MT_TRAIN), 0, st, D, N, X, Y, n_rows, idx, step, steps, S, lr,
                       adam_t, mode, loss_out);
    return hipGetLastError();
}

hipError_t mlp_launch_refresh(const MlpDev& D, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_refresh, dim3(D.n_members), dim3(MT), 0, st, D);
    return hipGetLastError();
}

// Per-member outputs of ij_mlp_predict_noalloc: a file-scope device array,
// one copy per GPU, alive until the process ends.  In host code `scratch`
// names a host-side stand-in, never the device memory: host code uses only
// the address mlp_static_scratch looks up.
static __device__ __align__(256) float scratch[kMlpStaticScratchFloats];

hipError_t mlp_static_scratch(float** ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static float* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<float*>(p);
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t mlp_launch_infer(const MlpDev& D, const MlpNorm& N, const float* X, int n, float* members, float* mean,
                            float* spread, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int per_block = kInferRows * (MT / 64);
    const int blocks = (n + per_block - 1) / per_block;
    hipLaunchKernelGGL(k_mlp_infer, dim3(blocks, D.n_members), dim3(MT), 0, st, D, N, X, n, members);
    if (mean && spread)
        hipLaunchKernelGGL(k_mlp_reduce, dim3((n * kMlpOut + 255) / 256), dim3(256), 0, st, members, D.n_members, n,
                           mean, spread);
    return hipGetLastError();
}

}  // namespace ij
