// lbm_core.h -- kernel parameter block and launchers of the binary-fluid
// lattice Boltzmann kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ij {

// Buffer layout: 14 float planes (f_0..f_8 shifted by w_i n0, then g_0..g_4)
// followed by one plane of 16-bit words holding the bfloat16 remainder
// g_0 - float(g_0) of the rest order-parameter population.
constexpr int kFloatPlanes = 14;

// Per-launch constants, derived on the host in double precision.  The
// order-parameter path (phi, ghosts, stencils, mu, force) runs in double,
// the collision of the distributions in float.
struct KParams {
    int nx, ny, pitch;
    int bc_open;          // 1: "fully developed" top and bottom rows
    int force_rows;       // body force on fluid nodes with y < force_rows
    unsigned plane;       // elements per plane (ny * pitch)
    // double-precision order-parameter constants
    double phi_star, beta4, kappa, gamma, omega_phi, inv_width;
    double wet[4];        // ghost offset 2 Omega phi*/W per wall class (index 1, 2)
    // float constants of the collision
    float n0, inv_phi_star, tau_amb, dtau, omq, c_half_q, omega_phi_f, gamma_f;
    float fb;             // body force of the current step (Fig. 1 pulse)
};

struct DiagRow {
    double mass_n, mass_phi, mom_x, mom_y, uy, max_u;
    int count, bad;
};

// Device record of one diagnostics sample; same layout as ij_sample.
struct SampleRec {
    int64_t step;
    double mass_n, mass_phi, mom_x, mom_y, max_u;
    int64_t nan_count, n_detached, largest_count;
    double largest_uy;
    int64_t largest_top;
};

hipError_t launch_phi_ghost(const KParams& P, const float* A, const uint8_t* wall, double* phi,
                            const int2* ghost_list, int n_ghost, hipStream_t st);
hipError_t launch_collide_ref(const KParams& P, const float* A, float* B, const uint8_t* wall,
                              const double* phi, hipStream_t st);
// plain_rows: [n_strips][ny] bytes, 1 where the row of the strip is plain
// (see the kernel).  The plain launch covers every tile of rows_per_block
// rows; general_tiles lists the tiles of rows_general rows (numbered
// block * n_strips + strip) that hold other rows.
hipError_t launch_collide_fused(const KParams& P, const float* A, float* B, const uint8_t* wall,
                                const uint8_t* plain_rows, const int* general_tiles, int n_general_tiles,
                                int waves_x, int rows_per_block, int rows_general, hipStream_t st);
hipError_t launch_init(const KParams& P, float* A, const uint8_t* wall, double* phi, const float* src,
                       int from_distance, const float* ux, const float* uy, const int2* ghost_list,
                       int n_ghost, hipStream_t st);
hipError_t launch_moments(const KParams& P, const float* A, const uint8_t* wall, const double* phi, float* n,
                          float* ph, float* ux, float* uy, hipStream_t st);
hipError_t launch_state_io(const KParams& P, float* A, float* f_ext, float* g_ext, int to_ext,
                           hipStream_t st);
hipError_t launch_diag(const KParams& P, const float* A, const uint8_t* wall, const double* phi, int row0,
                       int a_min, int64_t step, DiagRow* rows, SampleRec* out, hipStream_t st);

} // namespace ij
