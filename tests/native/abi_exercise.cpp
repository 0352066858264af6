// Host-side exercise of every entry point of the C ABI (include/inkjet_lbm.h),
// built with the host code under AddressSanitizer and UndefinedBehaviorSanitizer
// (device code is built as usual).  Each call is made with valid arguments and
// with the invalid ones its declaration documents (NULL handles and outputs,
// sizes out of range, a truncated or foreign checkpoint blob), so that the
// host logic behind them (parameter checks, the wall analysis, tile lists,
// graphs, the autotuners, checkpoint headers, the surrogate's packing) runs
// under the sanitizers.  Results are not checked here: the parity tests do
// that.  Prints one line per group and "abi_exercise: ok" at the end; exits 1
// on the first unexpected status.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "inkjet_lbm.h"

namespace {

int g_fail = 0;

void expect(const char* what, ij_status got, ij_status want)
{
    if (got != want) {
        std::fprintf(stderr, "abi_exercise: %s returned %d, expected %d\n", what, (int)got, (int)want);
        g_fail = 1;
        std::exit(1);
    }
}

#define OK(call) expect(#call, (call), IJ_OK)
#define BAD(call, code) expect(#call, (call), (code))

template <class T>
T* dev_alloc(size_t n)
{
    void* p = nullptr;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) {
        std::fprintf(stderr, "abi_exercise: hipMalloc of %zu bytes failed\n", n * sizeof(T));
        std::exit(1);
    }
    return static_cast<T*>(p);
}

template <class T>
T* dev_copy(const std::vector<T>& h)
{
    T* d = dev_alloc<T>(h.size());
    if (hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) std::exit(1);
    return d;
}

// a 96 x 128 lattice with a nozzle 24 wide and 32 long, a pulse and open rows
ij_params nozzle_params()
{
    ij_params p;
    ij_params_default(&p);
    p.nx = 96;
    p.ny = 128;
    p.bc_y = IJ_BC_OPEN;
    p.force_rows = 32;
    p.t_pos = 20;
    p.t_neg = 10;
    p.t_idle = 10;
    p.periodic_pulse = 1;
    p.nozzle_x0 = 36;
    p.nozzle_w = 24;
    p.nozzle_len = 32;
    p.diag_row0 = 32;
    p.diag_every = 10;
    p.tau_ink = 0.8;
    p.theta_inner = 60.0;
    p.theta_outer = 120.0;
    p.f_pos = 1e-4;
    p.f_neg = 5e-5;
    return p;
}

void exercise_single()
{
    ij_params p = nozzle_params();
    ij_sim* s = nullptr;
    ij_params bad = p;
    bad.nx = 2;
    BAD(ij_create(&bad, &s), IJ_ERR_INVALID_ARG);
    if (s != nullptr || std::strlen(ij_last_error(nullptr)) == 0) std::exit(1);
    BAD(ij_create(nullptr, &s), IJ_ERR_INVALID_ARG);
    bad = p;
    bad.tau_ink = 0.4;
    BAD(ij_create(&bad, &s), IJ_ERR_INVALID_ARG);
    size_t need = 0;
    OK(ij_required_bytes(&p, &need));
    OK(ij_create(&p, &s));
    BAD(ij_step(s, 1, nullptr), IJ_ERR_STATE);   // before init
    OK(ij_init_default(s, nullptr));
    OK(ij_step(s, 25, nullptr));
    BAD(ij_step(s, -1, nullptr), IJ_ERR_INVALID_ARG);
    OK(ij_step_reference(s, 3, nullptr));
    if (ij_time(s) != 28) std::exit(1);

    const size_t nodes = (size_t)p.nx * p.ny;
    float* n = dev_alloc<float>(nodes);
    float* phi = dev_alloc<float>(nodes);
    float* ux = dev_alloc<float>(nodes);
    float* uy = dev_alloc<float>(nodes);
    OK(ij_get_moments(s, n, phi, ux, uy, nullptr));
    OK(ij_get_moments(s, nullptr, phi, nullptr, uy, nullptr));   // outputs may be NULL
    float* f = dev_alloc<float>(9 * nodes);
    float* g = dev_alloc<float>(5 * nodes);
    OK(ij_get_state(s, f, g, nullptr));
    OK(ij_set_state(s, f, g, 28, nullptr));

    // checkpoint blob: whole, truncated, and with a damaged header
    size_t bytes = 0;
    OK(ij_state_bytes(s, &bytes));
    std::vector<unsigned char> blob(bytes);
    OK(ij_save_state(s, blob.data(), bytes, nullptr));
    BAD(ij_save_state(s, blob.data(), bytes - 1, nullptr), IJ_ERR_INVALID_ARG);
    OK(ij_load_state(s, blob.data(), bytes, nullptr));
    BAD(ij_load_state(s, blob.data(), bytes - 1, nullptr), IJ_ERR_INVALID_ARG);
    BAD(ij_load_state(s, blob.data(), 16, nullptr), IJ_ERR_INVALID_ARG);
    std::vector<unsigned char> damaged = blob;
    damaged[0] ^= 0xff;
    BAD(ij_load_state(s, damaged.data(), bytes, nullptr), IJ_ERR_INVALID_ARG);

    // diagnostics
    OK(ij_diag_sample(s, nullptr));
    std::vector<int64_t> count(p.ny);
    std::vector<double> uyr(p.ny);
    OK(ij_get_row_profile(s, count.data(), uyr.data(), nullptr));
    std::vector<ij_sample> smp(8);
    int64_t got = 0;
    OK(ij_get_samples(s, smp.data(), (int64_t)smp.size(), &got, nullptr));
    OK(ij_get_samples(s, smp.data(), 1, &got, nullptr));   // fewer than recorded
    ij_diag d;
    OK(ij_get_diagnostics(s, &d, nullptr));
    BAD(ij_get_diagnostics(s, nullptr, nullptr), IJ_ERR_INVALID_ARG);
    OK(ij_check(s, nullptr));
    double der[8];
    OK(ij_derived(s, der));

    // tile shapes, the autotuner, the wall from either side
    OK(ij_set_tiling(s, 2, 16));
    OK(ij_step(s, 7, nullptr));
    OK(ij_set_tiling(s, 4, 1));
    BAD(ij_set_tiling(s, 3, 1), IJ_ERR_INVALID_ARG);
    int32_t wx = 0, rows = 0;
    double ms = 0.0;
    OK(ij_autotune(s, 3, nullptr, &wx, &rows, &ms));
    OK(ij_autotune(s, 3, nullptr, nullptr, nullptr, nullptr));
    std::vector<uint8_t> wall(nodes, IJ_FLUID);
    for (int y = 0; y < 32; ++y)
        for (int x = 0; x < 96; ++x)
            if (x < 36 || x >= 60) wall[(size_t)y * 96 + x] = IJ_WALL_INNER;
    OK(ij_set_wall(s, wall.data()));
    uint8_t* wd = dev_copy(wall);
    OK(ij_set_solid_mask(s, wd, 1));
    OK(ij_set_solid_mask(s, wall.data(), 0));
    std::vector<uint8_t> wrong = wall;
    wrong[5] = 9;
    BAD(ij_set_wall(s, wrong.data()), IJ_ERR_INVALID_ARG);
    BAD(ij_set_solid_mask(s, nullptr, 1), IJ_ERR_INVALID_ARG);

    // initial states from device fields, then caller-owned buffers
    std::vector<float> dist(nodes);
    for (int y = 0; y < p.ny; ++y)
        for (int x = 0; x < p.nx; ++x) dist[(size_t)y * p.nx + x] = 40.5f - (float)y;
    float* dd = dev_copy(dist);
    OK(ij_init_distance(s, dd, nullptr));
    OK(ij_init_phi(s, dd, nullptr, nullptr, nullptr));
    OK(ij_step(s, 12, nullptr));
    void* a = dev_alloc<unsigned char>(need);
    void* b = dev_alloc<unsigned char>(need);
    BAD(ij_attach_buffers(s, a, b, need - 1), IJ_ERR_INVALID_ARG);
    OK(ij_attach_buffers(s, a, b, need));
    OK(ij_init_distance(s, dd, nullptr));
    OK(ij_step(s, 12, nullptr));
    if (hipDeviceSynchronize() != hipSuccess) std::exit(1);
    ij_destroy(s);
    ij_destroy(nullptr);
    for (void* q : {(void*)n, (void*)phi, (void*)ux, (void*)uy, (void*)f, (void*)g, (void*)wd, (void*)dd, a, b})
        (void)hipFree(q);
    std::printf("abi_exercise: single lattice ok\n");
}

void exercise_batch()
{
    std::vector<ij_params> cases;
    for (int k = 0; k < 3; ++k) {
        ij_params p = nozzle_params();
        p.nx = 80 + 40 * k;   // uneven widths: full strips and ragged tails
        p.nozzle_x0 = (p.nx - 24) / 2;
        p.theta_inner = 45.0 + 40.0 * k;
        cases.push_back(p);
    }
    ij_batch* b = nullptr;
    BAD(ij_batch_create(cases.data(), 0, &b), IJ_ERR_INVALID_ARG);
    OK(ij_batch_create(cases.data(), (int32_t)cases.size(), &b));
    if (ij_batch_size(b) != 3) std::exit(1);
    ij_sim* c = nullptr;
    OK(ij_batch_case(b, 1, &c));
    BAD(ij_batch_case(b, 3, &c), IJ_ERR_INVALID_ARG);
    for (int k = 0; k < 3; ++k) {
        OK(ij_batch_case(b, k, &c));
        OK(ij_init_default(c, nullptr));
    }
    BAD(ij_step(c, 1, nullptr), IJ_ERR_STATE);   // members step with their batch
    OK(ij_batch_step(b, 9, nullptr));
    OK(ij_batch_set_graph(b, 10));
    OK(ij_batch_step(b, 23, nullptr));
    int32_t w = 0, r = 0, m = 0, per = 0;
    OK(ij_batch_get_tiling(b, &w, &r, &m, &per));
    OK(ij_batch_set_tiling(b, 2, 1, 0, 0));
    OK(ij_batch_step(b, 5, nullptr));
    OK(ij_batch_set_tiling(b, 4, 32, 1, 1));
    OK(ij_batch_step(b, 5, nullptr));
    BAD(ij_batch_set_tiling(b, 5, 1, 0, 0), IJ_ERR_INVALID_ARG);
    double ms = 0.0;
    OK(ij_batch_autotune(b, 3, nullptr, &w, &r, &m, &per, &ms));
    OK(ij_batch_set_graph(b, 0));
    OK(ij_batch_step(b, 4, nullptr));
    if (ij_batch_time(b) != 46) std::exit(1);
    OK(ij_batch_case(b, 2, &c));
    size_t bytes = 0;
    OK(ij_state_bytes(c, &bytes));
    std::vector<unsigned char> blob(bytes);
    OK(ij_save_state(c, blob.data(), bytes, nullptr));
    ij_diag d;
    OK(ij_get_diagnostics(c, &d, nullptr));
    if (hipDeviceSynchronize() != hipSuccess) std::exit(1);
    ij_batch_destroy(b);
    ij_batch_destroy(nullptr);
    std::printf("abi_exercise: batch ok\n");
}

void exercise_mlp()
{
    ij_mlp* m = nullptr;
    BAD(ij_mlp_create(0, &m), IJ_ERR_INVALID_ARG);
    BAD(ij_mlp_create_seeded(65, 1, &m), IJ_ERR_INVALID_ARG);
    OK(ij_mlp_create_seeded(3, 77, &m));
    const int np = ij_mlp_param_count();
    std::vector<double> w(np);
    OK(ij_mlp_get_weights(m, 2, w.data()));
    BAD(ij_mlp_get_weights(m, 3, w.data()), IJ_ERR_INVALID_ARG);
    OK(ij_mlp_set_weights(m, 0, w.data()));
    std::vector<double> nanw = w;
    nanw[7] = NAN;
    BAD(ij_mlp_set_weights(m, 0, nanw.data()), IJ_ERR_INVALID_ARG);
    const double xm[7] = {90, 0.01, 1.5e-4, 1.5e-4, 1750, 1750, 1750};
    const double xs[7] = {35, 0.004, 7e-5, 7e-5, 700, 700, 700};
    const double ym[3] = {20000, 0.01, 5000}, ys[3] = {10000, 0.01, 3000};
    OK(ij_mlp_set_scaling(m, xm, xs, ym, ys));
    const int n = 300;
    std::vector<float> x(n * 7), y(n * 4);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < 7; ++j) x[i * 7 + j] = (float)(xm[j] + xs[j] * std::sin(0.37 * i + j));
        y[i * 4 + 0] = (float)(ym[0] + ys[0] * std::cos(0.11 * i));
        y[i * 4 + 1] = (float)(ym[1] + ys[1] * std::sin(0.05 * i));
        y[i * 4 + 2] = (float)(ym[2] + ys[2] * std::cos(0.07 * i));
        y[i * 4 + 3] = (float)(i % 3 == 0);
    }
    float* xd = dev_copy(x);
    float* yd = dev_copy(y);
    std::vector<double> grad((size_t)3 * np), loss(3);
    OK(ij_mlp_gradients(m, xd, yd, 64, grad.data(), loss.data(), nullptr));
    BAD(ij_mlp_gradients(m, xd, yd, 0, grad.data(), loss.data(), nullptr), IJ_ERR_INVALID_ARG);
    const int steps = 5, batch = 32;
    std::vector<int32_t> idx((size_t)3 * steps * batch);
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int32_t)((i * 7919u) % n);
    int32_t* idxd = dev_copy(idx);
    float* lossd = dev_alloc<float>(3 * steps);
    OK(ij_mlp_train(m, xd, yd, n, idxd, steps, batch, 1e-3f, lossd, nullptr));
    OK(ij_mlp_train(m, xd, yd, n, idxd, steps, batch, 1e-3f, nullptr, nullptr));
    BAD(ij_mlp_train(m, xd, yd, n, idxd, steps, 0, 1e-3f, nullptr, nullptr), IJ_ERR_INVALID_ARG);
    float* mean = dev_alloc<float>(n * 4);
    float* spread = dev_alloc<float>(n * 4);
    float* members = dev_alloc<float>(3 * n * 4);
    OK(ij_mlp_predict(m, xd, n, mean, spread, members, nullptr));
    OK(ij_mlp_predict(m, xd, n, mean, spread, nullptr, nullptr));
    OK(ij_mlp_predict(m, xd, 0, mean, spread, nullptr, nullptr));
    OK(ij_mlp_predict_noalloc(m, xd, n, mean, spread, nullptr));
    OK(ij_mlp_predict_noalloc(m, xd, 17, mean, spread, nullptr));
    BAD(ij_mlp_predict_noalloc(m, xd, 524288 / 3 + 1, mean, spread, nullptr), IJ_ERR_INVALID_ARG);
    BAD(ij_mlp_predict_noalloc(m, xd, n, nullptr, spread, nullptr), IJ_ERR_INVALID_ARG);
    if (hipDeviceSynchronize() != hipSuccess) std::exit(1);
    ij_mlp_destroy(m);
    ij_mlp_destroy(nullptr);
    for (void* q : {(void*)xd, (void*)yd, (void*)idxd, (void*)lossd, (void*)mean, (void*)spread, (void*)members})
        (void)hipFree(q);
    std::printf("abi_exercise: surrogate ok\n");
}

void exercise_3d()
{
    ij3_params p;
    std::memset(&p, 0, sizeof p);
    p.nx = 40;
    p.ny = 48;
    p.nz = 36;
    p.bc_y = IJ_BC_OPEN;
    p.force_rows = 12;
    p.t_pos = 10;
    p.t_neg = 5;
    p.t_idle = 5;
    p.periodic_pulse = 1;
    p.rho_ink = 1.0;
    p.rho_amb = 0.1;
    p.sigma = 0.01;
    p.width = 4.0;
    p.gamma = 1.0;
    p.tau_ink = 0.8;
    p.tau_amb = 1.0;
    p.tau_phi = 1.0;
    p.theta_inner = 60.0;
    p.theta_outer = 120.0;
    p.f_pos = 1e-4;
    p.f_neg = 5e-5;
    const size_t nodes = (size_t)p.nx * p.ny * p.nz;
    // a round bore of radius 8 through the first 12 rows
    std::vector<uint8_t> wall(nodes, IJ_FLUID);
    for (int y = 0; y < 12; ++y)
        for (int z = 0; z < p.nz; ++z)
            for (int x = 0; x < p.nx; ++x) {
                const double r = std::hypot(x - 19.5, z - 17.5);
                if (r > 8.0) wall[((size_t)y * p.nz + z) * p.nx + x] = IJ_WALL_INNER;
            }
    ij3_sim* s = nullptr;
    ij3_params bad = p;
    bad.nz = 2;
    BAD(ij3_create(&bad, wall.data(), &s), IJ_ERR_INVALID_ARG);
    OK(ij3_create(&p, wall.data(), &s));
    std::vector<float> dist(nodes);
    for (int y = 0; y < p.ny; ++y)
        for (size_t k = 0; k < (size_t)p.nz * p.nx; ++k) dist[(size_t)y * p.nz * p.nx + k] = 14.5f - (float)y;
    float* dd = dev_copy(dist);
    OK(ij3_init(s, dd, 1, nullptr, nullptr, nullptr, nullptr));
    BAD(ij3_init(s, nullptr, 1, nullptr, nullptr, nullptr, nullptr), IJ_ERR_INVALID_ARG);
    OK(ij3_step(s, 9, nullptr));
    if (ij3_time(s) != 9) std::exit(1);
    float* mo[5];
    for (auto& q : mo) q = dev_alloc<float>(nodes);
    OK(ij3_get_moments(s, mo[0], mo[1], mo[2], mo[3], mo[4], nullptr));
    float* f = dev_alloc<float>(19 * nodes);
    float* g = dev_alloc<float>(7 * nodes);
    OK(ij3_get_state(s, f, g, nullptr));
    OK(ij3_set_state(s, f, g, 9, nullptr));
    size_t bytes = 0;
    OK(ij3_state_bytes(s, &bytes));
    std::vector<unsigned char> blob(bytes);
    OK(ij3_save_state(s, blob.data(), bytes, nullptr));
    OK(ij3_load_state(s, blob.data(), bytes, nullptr));
    BAD(ij3_load_state(s, blob.data(), bytes / 2, nullptr), IJ_ERR_INVALID_ARG);
    double rec[7];
    std::vector<int64_t> cnt(p.ny);
    std::vector<double> uy(p.ny);
    ij3_drops drops;
    OK(ij3_sample(s, 12, rec, cnt.data(), uy.data(), 4, 2, &drops, nullptr));
    OK(ij3_sample(s, 12, rec, nullptr, nullptr, 4, 2, nullptr, nullptr));
    OK(ij3_step(s, 3, nullptr));
    if (hipDeviceSynchronize() != hipSuccess) std::exit(1);
    ij3_destroy(s);
    ij3_destroy(nullptr);
    for (auto q : mo) (void)hipFree(q);
    (void)hipFree(f);
    (void)hipFree(g);
    (void)hipFree(dd);
    std::printf("abi_exercise: three-dimensional lattice ok\n");
}

}  // namespace

int main()
{
    exercise_single();
    exercise_batch();
    exercise_mlp();
    exercise_3d();
    std::printf("abi_exercise: ok\n");
    return g_fail;
}
