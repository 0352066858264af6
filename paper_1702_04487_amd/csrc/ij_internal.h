// ij_internal.h -- host-side state of a simulation handle and the helpers
// shared by the single-lattice API (ij_api.cpp) and batches (ij_batch.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "checkpoint.h"
#include "inkjet_lbm.h"
#include "lbm_core.h"

namespace ij_host {

using ij_ckpt::StateHeader;
using ij_ckpt::fnv1a;

constexpr int kPitchAlign = 64;    // floats: 256-byte rows
constexpr int64_t kSampleCap = 4096;
// rows per tile of the launch over rows next to solid nodes: short tiles
// when such rows are few and scattered (many workgroups, little marching),
// taller ones when a strip has long runs of them (less pipeline overhead)
constexpr int kGeneralRowsShort = 4, kGeneralRowsTall = 8, kGeneralTallRun = 32;

inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// one distribution buffer: 14 float planes and the 16-bit g_0 remainder plane
inline size_t buffer_bytes(size_t plane)
{
    return plane * (ij::kFloatPlanes * sizeof(float) + sizeof(uint16_t));
}

}  // namespace ij_host

struct ij_sim {
    ij_params p{};
    int nx = 0, ny = 0, pitch = 0;
    size_t plane = 0;  // floats per plane
    double phi_star = 0, n0 = 0, beta = 0, kappa = 0, q = 0, wet_in = 0, wet_out = 0;
    ij::KParams K{};
    float* buf[2] = {nullptr, nullptr};
    bool own[2] = {false, false};
    int cur = 0;
    uint8_t* wall = nullptr;   // device [ny][pitch]
    std::vector<uint8_t> wall_host;  // [ny][nx]
    double* phi = nullptr;     // device phi~ field [ny][pitch] (double)
    int2* ghost = nullptr;     // solid nodes that touch fluid
    int n_ghost = 0;
    ij::DiagRow* rows = nullptr;
    ij::SampleRec* samples = nullptr;  // device ring of kSampleCap
    int64_t n_dev_samples = 0;         // recorded on the device, not yet drained
    std::vector<ij_sample> host_samples;
    int64_t t = 0;
    bool initialised = false;
    int64_t unstable_step = -1;
    int waves_x = 4, rows_per_block = 1;   // 1: plain rows by the row kernel
    // rows of each strip the plain collide-stream path may take, and the
    // tiles that hold the other rows (rebuilt with the wall or the tiling)
    uint8_t* plain = nullptr;
    int4* gtiles = nullptr;            // (strip, block, first column, 0) of the general launch
    ij::DiagRow* sample_parts = nullptr;   // [ceil(nx/64)][ny] partials of a fused sample (on first use)
    int4* ptiles = nullptr;            // plain tiles that hold a plain row (when listed)
    int n_ptiles = -1;                 // their count; -1: the plain launch covers every tile
    int n_gtiles = 0;
    std::vector<int4> gtiles_host;
    std::vector<uint8_t> plain_host;   // the plain-row table [n_strips][ny] as uploaded
    std::vector<int> strip_x0;         // first column of each strip
    std::vector<uint8_t> tile_plain;   // per (row block, strip) tile: holds a plain row
    int n_strips = 0, n_rb = 0;   // of the plain launch's tiling
    int n_wide = 0;               // strips 64 * waves_x wide; the others are 64 wide
    bool mixed_strips = false;    // tail strips of 64 columns (batches)
    bool in_batch = false;        // owned and stepped by an ij_batch
    std::string err;
};

namespace ij_host {

ij_status fail(ij_sim* s, ij_status st, const std::string& msg);
ij_status hip_fail(ij_sim* s, hipError_t e, const char* where);
double pulse_value(const ij_params& p, int64_t t);
std::string validate(const ij_params& p);
ij_status build_plain(ij_sim* s);
ij_status drain_samples(ij_sim* s, hipStream_t st);
double u_limit(const ij_params& p);
// rows of the head and of the tail of a drop (one interface width)
int diag_band(double width);
void destroy_sim(ij_sim* s);   // frees a handle whatever its owner

}  // namespace ij_host
