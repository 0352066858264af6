// mlp_core.h -- layouts, device state and launchers of the surrogate network
// (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ij {

constexpr int kMlpIn = 7, kMlpHidden = 128, kMlpOut = 4, kMlpReg = 3;
constexpr int kMlpMaxBatch = 1024;   // rows of one training step

// padded float32 parameters of one member (offsets in floats)
constexpr int kMlpW1 = 0, kMlpW1Size = 128 * 16;
constexpr int kMlpB1 = kMlpW1 + kMlpW1Size;
constexpr int kMlpW2 = kMlpB1 + 128, kMlpW2Size = 128 * 128;
constexpr int kMlpB2 = kMlpW2 + kMlpW2Size;
constexpr int kMlpW3 = kMlpB2 + 128, kMlpW3Size = 16 * 128;
constexpr int kMlpB3 = kMlpW3 + kMlpW3Size;
constexpr int kMlpParams = kMlpB3 + 16;
// bfloat16 copies of the weight matrices (offsets in elements)
constexpr int kMlpW1b = 0, kMlpW2b = kMlpW1Size, kMlpW3b = kMlpW1Size + kMlpW2Size;
constexpr int kMlpWeightsBf16 = kMlpW3b + kMlpW3Size;
// unpadded parameter count (W1 128x7, b1, W2 128x128, b2, W3 4x128, b3)
constexpr int kMlpPacked = 128 * 7 + 128 + 128 * 128 + 128 + 4 * 128 + 4;

// input and target scaling: x_n = (x - x_mean) * x_inv_std, regression
// targets t_n = (y - y_mean) * y_inv_std and y = o * y_std + y_mean
struct MlpNorm {
    float x_mean[kMlpIn], x_inv_std[kMlpIn];
    float y_mean[kMlpReg], y_inv_std[kMlpReg], y_std[kMlpReg];
};

struct MlpDev {
    int n_members;
    float* w;        // [members][kMlpParams] master parameters
    float* m;        // Adam moments
    float* v;
    float* g;        // gradients
    uint16_t* wb;    // [members][kMlpWeightsBf16]
    uint8_t* scratch;
    size_t scratch_per_member;
};

// per-member activations and gradients of one training step (kMlpMaxBatch rows)
struct MlpScratch {
    uint16_t* xn;   // [B][16]
    float* z1;      // [B][128]
    uint16_t* a1;
    float* z2;
    uint16_t* a2;
    float* dof;     // [B][16]
    uint16_t* dob;
    float* dzf;     // dZ2 [B][128]
    uint16_t* dzb;
    float* dz1f;    // dZ1 [B][128]
    uint16_t* dz1b;
};

__host__ __device__ inline size_t mlp_align(size_t v) { return (v + 255) & ~(size_t)255; }

__host__ __device__ inline size_t mlp_scratch_bytes()
{
    const size_t B = kMlpMaxBatch;
    return mlp_align(B * 16 * 2) + 2 * mlp_align(B * 128 * 4) + 2 * mlp_align(B * 128 * 2) + mlp_align(B * 16 * 4) +
           mlp_align(B * 16 * 2) + 2 * mlp_align(B * 128 * 4) + 2 * mlp_align(B * 128 * 2);
}

__host__ __device__ inline MlpScratch mlp_scratch(const MlpDev& D, int member)
{
    const size_t B = kMlpMaxBatch;
    uint8_t* p = D.scratch + (size_t)member * D.scratch_per_member;
    MlpScratch s;
    auto take = [&](size_t bytes) {
        uint8_t* r = p;
        p += mlp_align(bytes);
        return r;
    };
    s.xn = (uint16_t*)take(B * 16 * 2);
    s.z1 = (float*)take(B * 128 * 4);
    s.a1 = (uint16_t*)take(B * 128 * 2);
    s.z2 = (float*)take(B * 128 * 4);
    s.a2 = (uint16_t*)take(B * 128 * 2);
    s.dof = (float*)take(B * 16 * 4);
    s.dob = (uint16_t*)take(B * 16 * 2);
    s.dzf = (float*)take(B * 128 * 4);
    s.dzb = (uint16_t*)take(B * 128 * 2);
    s.dz1f = (float*)take(B * 128 * 4);
    s.dz1b = (uint16_t*)take(B * 128 * 2);
    return s;
}

// one training step of every member (mode 0: gradients + Adam step adam_t;
// mode 1: gradients only); rows idx[member][step][0..S) (clamped to [0, n_rows))
// or 0..S-1 (idx null)
hipError_t mlp_launch_step(const MlpDev& D, const MlpNorm& N, const float* X, const float* Y, int n_rows,
                           const int* idx, int step, int steps, int S, float lr, int adam_t, int mode,
                           float* loss_out, hipStream_t st);
hipError_t mlp_launch_refresh(const MlpDev& D, hipStream_t st);
// members [n_members][n][4]; mean and spread [n][4] when both are given
hipError_t mlp_launch_infer(const MlpDev& D, const MlpNorm& N, const float* X, int n, float* members, float* mean,
                            float* spread, hipStream_t st);

// Floats of the fixed per-device scratch array of the prediction that
// allocates nothing (8 MiB: the per-member outputs of n * n_members <=
// 524288 query-member pairs).
constexpr size_t kMlpStaticScratchFloats = (size_t)1 << 21;
// Device address of that array on the current device: looked up with
// hipGetSymbolAddress on the first call for each device (with that device
// current) and kept for the life of the process.  No allocation.
hipError_t mlp_static_scratch(float** ptr);

}  // namespace ij
