// ij_mlp.cpp -- C ABI of the surrogate network (include/inkjet_lbm.h):
// parameters in and out, input/target scaling, training steps, gradients and
// ensemble prediction.  All arithmetic of the network runs in mlp.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "inkjet_lbm.h"
#include "mlp_core.h"

using namespace ij;

namespace {
thread_local std::string g_mlp_create_error;
}

struct ij_mlp {
    MlpDev D{};
    MlpNorm N{};
    int device = 0;           // the device that holds the parameters
    int64_t adam_steps = 0;   // Adam steps taken since the parameters were set
    float* members = nullptr; // prediction scratch [n_members][cap][4]
    int64_t members_cap = 0;
    std::string err;
};

namespace {

ij_status mfail(ij_mlp* m, ij_status st, const std::string& msg)
{
    if (m)
        m->err = msg;
    else
        g_mlp_create_error = msg;
    return st;
}

ij_status mhip(ij_mlp* m, hipError_t e, const char* where)
{
    return mfail(m, IJ_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define IJM_HIP(m, call)                                   \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return mhip(m, e_, #call);   \
    } while (0)

// packed (W1 128x7, b1, W2 128x128, b2, W3 4x128, b3) <-> padded layout
void unpack(const double* src, float* w)
{
    std::memset(w, 0, sizeof(float) * kMlpParams);
    const double* p = src;
    for (int o = 0; o < 128; ++o)
        for (int i = 0; i < kMlpIn; ++i) w[kMlpW1 + o * 16 + i] = (float)*p++;
    for (int o = 0; o < 128; ++o) w[kMlpB1 + o] = (float)*p++;
    for (int o = 0; o < 128; ++o)
        for (int i = 0; i < 128; ++i) w[kMlpW2 + o * 128 + i] = (float)*p++;
    for (int o = 0; o < 128; ++o) w[kMlpB2 + o] = (float)*p++;
    for (int o = 0; o < kMlpOut; ++o)
        for (int i = 0; i < 128; ++i) w[kMlpW3 + o * 128 + i] = (float)*p++;
    for (int o = 0; o < kMlpOut; ++o) w[kMlpB3 + o] = (float)*p++;
}

void pack(const float* w, double* dst)
{
    double* p = dst;
    for (int o = 0; o < 128; ++o)
        for (int i = 0; i < kMlpIn; ++i) *p++ = w[kMlpW1 + o * 16 + i];
    for (int o = 0; o < 128; ++o) *p++ = w[kMlpB1 + o];
    for (int o = 0; o < 128; ++o)
        for (int i = 0; i < 128; ++i) *p++ = w[kMlpW2 + o * 128 + i];
    for (int o = 0; o < 128; ++o) *p++ = w[kMlpB2 + o];
    for (int o = 0; o < kMlpOut; ++o)
        for (int i = 0; i < 128; ++i) *p++ = w[kMlpW3 + o * 128 + i];
    for (int o = 0; o < kMlpOut; ++o) *p++ = w[kMlpB3 + o];
}

}  // namespace

extern "C" {

ij_status ij_mlp_create(int32_t n_members, ij_mlp** out)
{
    if (!out) return mfail(nullptr, IJ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_members < 1 || n_members > 64) return mfail(nullptr, IJ_ERR_INVALID_ARG, "n_members must lie in [1, 64]");
    ij_mlp* m = new ij_mlp();
    m->D.n_members = n_members;
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return mfail(nullptr, IJ_ERR_DEVICE, "hipGetDevice failed");
    }
    m->D.scratch_per_member = mlp_scratch_bytes();
    const size_t np = (size_t)n_members * kMlpParams * sizeof(float);
    if (hipMalloc(&m->D.w, np) != hipSuccess || hipMalloc(&m->D.m, np) != hipSuccess ||
        hipMalloc(&m->D.v, np) != hipSuccess || hipMalloc(&m->D.g, np) != hipSuccess ||
        hipMalloc(&m->D.wb, (size_t)n_members * kMlpWeightsBf16 * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&m->D.scratch, (size_t)n_members * m->D.scratch_per_member) != hipSuccess) {
        ij_mlp_destroy(m);
        return mfail(nullptr, IJ_ERR_OOM, "network allocation failed");
    }
    if (hipMemset(m->D.w, 0, np) != hipSuccess || hipMemset(m->D.m, 0, np) != hipSuccess ||
        hipMemset(m->D.v, 0, np) != hipSuccess || hipMemset(m->D.g, 0, np) != hipSuccess ||
        hipMemset(m->D.wb, 0, (size_t)n_members * kMlpWeightsBf16 * sizeof(uint16_t)) != hipSuccess) {
        ij_mlp_destroy(m);
        return mfail(nullptr, IJ_ERR_DEVICE, "hipMemset failed");
    }
    for (int i = 0; i < kMlpIn; ++i) m->N.x_inv_std[i] = 1.f;
    for (int i = 0; i < kMlpReg; ++i) m->N.y_inv_std[i] = m->N.y_std[i] = 1.f;
    *out = m;
    return IJ_OK;
}

void ij_mlp_destroy(ij_mlp* m)
{
    if (!m) return;
    (void)hipDeviceSynchronize();
    if (m->D.w) (void)hipFree(m->D.w);
    if (m->D.m) (void)hipFree(m->D.m);
    if (m->D.v) (void)hipFree(m->D.v);
    if (m->D.g) (void)hipFree(m->D.g);
    if (m->D.wb) (void)hipFree(m->D.wb);
    if (m->D.scratch) (void)hipFree(m->D.scratch);
    if (m->members) (void)hipFree(m->members);
    delete m;
}

const char* ij_mlp_last_error(const ij_mlp* m) { return m ? m->err.c_str() : g_mlp_create_error.c_str(); }

int32_t ij_mlp_param_count(void) { return kMlpPacked; }

ij_status ij_mlp_create_seeded(int32_t n_members, uint64_t seed, ij_mlp** out)
{
    ij_status r = ij_mlp_create(n_members, out);
    if (r != IJ_OK) return r;
    // member k: draw j of SplitMix64 (Steele, Lea & Flood 2014) started at
    // seed + 1000 k gives packed parameter j, uniform in +-1/sqrt(fan_in)
    // of its layer (u = top 53 bits / 2^53)
    std::vector<double> packed(kMlpParams);
    const int fan_in[3] = {kMlpIn, kMlpHidden, kMlpHidden};
    const int fan_out[3] = {kMlpHidden, kMlpHidden, kMlpOut};
    for (int k = 0; k < n_members; ++k) {
        const uint64_t s0 = seed + 1000ull * (uint64_t)k;
        size_t j = 0;
        for (int l = 0; l < 3; ++l) {
            const double a = 1.0 / std::sqrt((double)fan_in[l]);
            const size_t count = (size_t)fan_out[l] * fan_in[l] + fan_out[l];   // W then b
            for (size_t c = 0; c < count; ++c, ++j) {
                uint64_t z = s0 + (uint64_t)(j + 1) * 0x9E3779B97F4A7C15ull;
                z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
                z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
                z ^= z >> 31;
                const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
                const double span = (a - -a) * u;   // two statements: no fused multiply-add
                packed[j] = -a + span;
            }
        }
        r = ij_mlp_set_weights(*out, k, packed.data());
        if (r != IJ_OK) {
            ij_mlp_destroy(*out);
            *out = nullptr;
            return r;
        }
    }
    return IJ_OK;
}

ij_status ij_mlp_set_weights(ij_mlp* m, int32_t member, const double* packed)
{
    if (!m || !packed) return IJ_ERR_INVALID_ARG;
    if (member < 0 || member >= m->D.n_members) return mfail(m, IJ_ERR_INVALID_ARG, "member out of range");
    std::vector<float> w(kMlpParams);
    unpack(packed, w.data());
    for (float v : w)
        if (!std::isfinite(v)) return mfail(m, IJ_ERR_INVALID_ARG, "non-finite parameter");
    const size_t off = (size_t)member * kMlpParams;
    IJM_HIP(m, hipMemcpy(m->D.w + off, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice));
    IJM_HIP(m, hipMemset(m->D.m + off, 0, w.size() * sizeof(float)));
    IJM_HIP(m, hipMemset(m->D.v + off, 0, w.size() * sizeof(float)));
    IJM_HIP(m, mlp_launch_refresh(m->D, nullptr));
    IJM_HIP(m, hipDeviceSynchronize());
    m->adam_steps = 0;
    return IJ_OK;
}

ij_status ij_mlp_get_weights(ij_mlp* m, int32_t member, double* packed)
{
    if (!m || !packed) return IJ_ERR_INVALID_ARG;
    if (member < 0 || member >= m->D.n_members) return mfail(m, IJ_ERR_INVALID_ARG, "member out of range");
    std::vector<float> w(kMlpParams);
    IJM_HIP(m, hipDeviceSynchronize());
    IJM_HIP(m, hipMemcpy(w.data(), m->D.w + (size_t)member * kMlpParams, w.size() * sizeof(float),
                         hipMemcpyDeviceToHost));
    pack(w.data(), packed);
    return IJ_OK;
}

ij_status ij_mlp_set_scaling(ij_mlp* m, const double* x_mean, const double* x_std, const double* y_mean,
                             const double* y_std)
{
    if (!m || !x_mean || !x_std || !y_mean || !y_std) return IJ_ERR_INVALID_ARG;
    for (int i = 0; i < kMlpIn; ++i)
        if (!(x_std[i] > 0.0) || !std::isfinite(x_mean[i])) return mfail(m, IJ_ERR_INVALID_ARG, "bad input scaling");
    for (int i = 0; i < kMlpReg; ++i)
        if (!(y_std[i] > 0.0) || !std::isfinite(y_mean[i])) return mfail(m, IJ_ERR_INVALID_ARG, "bad target scaling");
    for (int i = 0; i < kMlpIn; ++i) {
        m->N.x_mean[i] = (float)x_mean[i];
        m->N.x_inv_std[i] = (float)(1.0 / x_std[i]);
    }
    for (int i = 0; i < kMlpReg; ++i) {
        m->N.y_mean[i] = (float)y_mean[i];
        m->N.y_inv_std[i] = (float)(1.0 / y_std[i]);
        m->N.y_std[i] = (float)y_std[i];
    }
    return IJ_OK;
}

ij_status ij_mlp_gradients(ij_mlp* m, const float* x_dev, const float* y_dev, int32_t n, double* grad, double* loss,
                           void* stream)
{
    if (!m || !x_dev || !y_dev || !grad) return IJ_ERR_INVALID_ARG;
    if (n < 1 || n > kMlpMaxBatch) return mfail(m, IJ_ERR_INVALID_ARG, "n must lie in [1, 1024]");
    hipStream_t st = (hipStream_t)stream;
    float* dloss = nullptr;
    IJM_HIP(m, hipMalloc(&dloss, sizeof(float) * m->D.n_members));
    hipError_t e = mlp_launch_step(m->D, m->N, x_dev, y_dev, n, nullptr, 0, 1, n, 0.f, 1, 1, dloss, st);
    std::vector<float> g((size_t)m->D.n_members * kMlpParams), l((size_t)m->D.n_members);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g.data(), m->D.g, g.size() * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(l.data(), dloss, l.size() * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dloss);
    if (e != hipSuccess) return mhip(m, e, "gradient kernels");
    for (int k = 0; k < m->D.n_members; ++k) {
        pack(g.data() + (size_t)k * kMlpParams, grad + (size_t)k * kMlpPacked);
        if (loss) loss[k] = l[(size_t)k];
    }
    return IJ_OK;
}

ij_status ij_mlp_train(ij_mlp* m, const float* x_dev, const float* y_dev, int32_t n_rows, const int32_t* idx_dev,
                       int32_t steps, int32_t batch, float lr, float* loss_dev, void* stream)
{
    if (!m || !x_dev || !y_dev || !idx_dev) return IJ_ERR_INVALID_ARG;
    if (n_rows < 1) return mfail(m, IJ_ERR_INVALID_ARG, "n_rows must be >= 1");
    if (batch < 1 || batch > kMlpMaxBatch) return mfail(m, IJ_ERR_INVALID_ARG, "batch must lie in [1, 1024]");
    if (steps < 0) return mfail(m, IJ_ERR_INVALID_ARG, "steps < 0");
    if (!(lr > 0.f) || !std::isfinite(lr)) return mfail(m, IJ_ERR_INVALID_ARG, "lr must be positive");
    hipStream_t st = (hipStream_t)stream;
    for (int32_t s = 0; s < steps; ++s) {
        const hipError_t e = mlp_launch_step(m->D, m->N, x_dev, y_dev, n_rows, idx_dev, s, steps, batch, lr,
                                             (int)(m->adam_steps + 1), 0, loss_dev, st);
        if (e != hipSuccess) return mhip(m, e, "training step kernel");
        ++m->adam_steps;
    }
    return IJ_OK;
}

ij_status ij_mlp_predict(ij_mlp* m, const float* x_dev, int64_t n, float* mean_dev, float* spread_dev,
                         float* members_dev, void* stream)
{
    if (!m || !x_dev) return IJ_ERR_INVALID_ARG;
    if (n < 0 || n > (int64_t)1 << 28) return mfail(m, IJ_ERR_INVALID_ARG, "n out of range");
    if (!members_dev && !(mean_dev && spread_dev))
        return mfail(m, IJ_ERR_INVALID_ARG, "need mean and spread, or the per-member outputs");
    if (n == 0) return IJ_OK;
    float* mem = members_dev;
    if (!mem) {
        if (n > m->members_cap) {
            if (m->members) (void)hipFree(m->members);
            m->members = nullptr;
            m->members_cap = 0;
            if (hipMalloc(&m->members, (size_t)n * m->D.n_members * kMlpOut * sizeof(float)) != hipSuccess)
                return mfail(m, IJ_ERR_OOM, "prediction scratch allocation failed");
            m->members_cap = n;
        }
        mem = m->members;
    }
    const hipError_t e = mlp_launch_infer(m->D, m->N, x_dev, (int)n, mem, mean_dev, spread_dev, (hipStream_t)stream);
    return e == hipSuccess ? IJ_OK : mhip(m, e, "inference kernels");
}

ij_status ij_mlp_predict_noalloc(ij_mlp* m, const float* x_dev, int64_t n, float* mean_dev, float* spread_dev,
                                 void* stream)
{
    if (!m) return IJ_ERR_INVALID_ARG;
    if (n == 0) return IJ_OK;
    if (!x_dev || !mean_dev || !spread_dev) return mfail(m, IJ_ERR_INVALID_ARG, "x, mean and spread are required");
    const int64_t max_n = (int64_t)(kMlpStaticScratchFloats / ((size_t)m->D.n_members * kMlpOut));
    if (n < 0 || n > max_n)
        return mfail(m, IJ_ERR_INVALID_ARG,
                     "n must lie in [0, " + std::to_string(max_n) + "]: the fixed scratch holds " +
                         std::to_string(kMlpStaticScratchFloats / kMlpOut) + " query-member outputs");
    int dev = -1;
    IJM_HIP(m, hipGetDevice(&dev));
    if (dev != m->device) return mfail(m, IJ_ERR_STATE, "the current device is not the handle's device");
    float* scratch_dev = nullptr;
    IJM_HIP(m, mlp_static_scratch(&scratch_dev));
    const hipError_t e =
        mlp_launch_infer(m->D, m->N, x_dev, (int)n, scratch_dev, mean_dev, spread_dev, (hipStream_t)stream);
    return e == hipSuccess ? IJ_OK : mhip(m, e, "inference kernels");
}

}  // extern "C"
