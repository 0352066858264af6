// lbm_core.h -- kernel parameter block and launchers of the binary-fluid
// lattice Boltzmann kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ij {

// Buffer layout: per lattice row, a block of 14 rows of pitch floats (f_0..f_8
// shifted by w_i n0, then g_0..g_4) and one row of pitch 16-bit words holding
// the bfloat16 remainder g_0 - float(g_0) of the rest order-parameter
// population; population i of node (x, y) is at y rs + i pitch + x with
// rs = 14.5 pitch floats.
constexpr int kFloatPlanes = 14;
constexpr int kMaxRowsPerBlock = 1024;   // rows of one tile (LDS row flags)

// Per-launch constants, derived on the host in double precision.  The
// order-parameter path (phi, ghosts, stencils, mu, force) runs in double,
// the collision of the distributions in float.
struct KParams {
    int nx, ny, pitch;
    int bc_open;          // 1: "fully developed" top and bottom rows
    int force_rows;       // body force on fluid nodes with y < force_rows
    int diag_row0;        // rows y >= diag_row0 count ink in a diagnostics sample
    unsigned plane;       // nodes of a padded lattice (ny * pitch): the size of the
                          // wall mask and the phi field
    unsigned rs;          // floats per lattice row of a buffer (14.5 * pitch)
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
    int64_t largest_bottom;
    double head_uy, tail_uy;
};

// One lattice of a batch as the batched kernels see it (device memory).
struct CaseRec {
    KParams P;              // P.fb: the body force of the current step (set on the device)
    float* buf[2];          // distribution buffers; buf[0] holds the state at parity 0
    const uint8_t* wall;    // [ny][pitch]
    const uint8_t* plain;   // plain-row table [n_strips][ny]
    DiagRow* parts;         // sample partials [ceil(nx/64)][ny] of a sampling step
    DiagRow* rows;          // [ny]
    SampleRec* ring;        // diagnostics records
    int row0, a_min, band;
    int64_t t_pos, t_neg, t_idle;
    int periodic;
    double f_pos, f_neg, u_limit;
};

hipError_t launch_phi_ghost(const KParams& P, const float* A, const uint8_t* wall, double* phi,
                            const int2* ghost_list, int n_ghost, hipStream_t st);
hipError_t launch_collide_ref(const KParams& P, const float* A, float* B, const uint8_t* wall,
                              const double* phi, hipStream_t st);
// plain_rows: [n_strips][ny] bytes, 1 where the row of the strip is plain
// (see the kernel).  The plain launch covers the tiles of rows_per_block
// rows of the strips of 64 * waves_x columns: every tile when n_plain_tiles
// is negative, else the n_plain_tiles (strip, first row, first column, rows)
// tiles listed in plain_tiles, row-block major (those that hold a plain
// row).  general_tiles lists the (strip, first row, first column, rows)
// pieces, 64 columns wide and at most kMaxRowsPerBlock rows, that hold the
// other rows.
// With sample_parts non-null the step also takes the diagnostics sample of
// its input state: one DiagRow per 64-column piece and row, [ceil(nx/64)][ny]
// (pieces without a fluid node are left untouched: clear them first).
hipError_t launch_collide_fused(const KParams& P, const float* A, float* B, const uint8_t* wall,
                                const uint8_t* plain_rows, const int4* plain_tiles, int n_plain_tiles,
                                const int4* general_tiles, int n_general_tiles, int waves_x, int rows_per_block,
                                DiagRow* sample_parts, hipStream_t st);
// Sample partials: clear n of them; sum them per row in a fixed order (n_sub
// pieces per row) into rows[ny] and reduce the rows to the record *out as
// launch_diag does.
hipError_t launch_sample_clear(DiagRow* parts, size_t n, hipStream_t st);
hipError_t launch_sample_finish(const DiagRow* parts, int n_sub, int ny, int row0, int a_min, int band,
                                int64_t step, DiagRow* rows, SampleRec* out, hipStream_t st);
hipError_t launch_init(const KParams& P, float* A, const uint8_t* wall, double* phi, const float* src,
                       int from_distance, const float* ux, const float* uy, const int2* ghost_list,
                       int n_ghost, hipStream_t st);
hipError_t launch_moments(const KParams& P, const float* A, const uint8_t* wall, const double* phi, float* n,
                          float* ph, float* ux, float* uy, hipStream_t st);
hipError_t launch_state_io(const KParams& P, float* A, const uint8_t* wall, float* f_ext, float* g_ext, int to_ext,
                           hipStream_t st);
hipError_t launch_diag(const KParams& P, const float* A, const uint8_t* wall, const double* phi, int row0,
                       int a_min, int band, int64_t step, DiagRow* rows, SampleRec* out, hipStream_t st);

// (case, strip, first row | rows << 16, first column) tiles of a batch:
// plain tiles of the wide strips (workgroups of 64 * waves_x lanes) and of
// the 64-column tail strips (one wave), and the 64-column general pieces
// (one wave); at most kMaxRowsPerBlock rows each.  The plain launches run
// grid_wide / grid_tail workgroups, each over a contiguous run of tiles (a
// grid of one workgroup per tile when it equals the tile count).
// With rows_per_block 1 the plain rows go to pieces (case, row, first column,
// nodes) of 64 columns of the plain strips of each row, one wave each and
// waves_x per workgroup, instead of walked plain tiles (n_wide = n_tail = 0).
struct BatchTiles {
    const int4 *wide, *tail, *gen, *rows;
    int n_wide, n_tail, n_gen, n_rows;
    int grid_wide, grid_tail;
};
// With sample, the step also takes each case's diagnostics sample of its
// input state into the case's partials (cleared before by
// launch_batch_sample_begin, reduced after by launch_batch_sample_end).
hipError_t launch_batch_collide(const BatchTiles& T, const CaseRec* cases, int parity, const int* active,
                                int waves_x, bool sample, hipStream_t st);
// the two halves of launch_batch_collide: the row pieces of the plain rows,
// and the rest (walked plain tiles, general pieces); independent of each
// other within a step
hipError_t launch_batch_rows(const BatchTiles& T, const CaseRec* cases, int parity, const int* active, int waves_x,
                             bool sample, hipStream_t st);
hipError_t launch_batch_general(const BatchTiles& T, const CaseRec* cases, int parity, const int* active,
                                int waves_x, bool sample, hipStream_t st);
// advances the step counter; a case switched off has its two buffers swapped,
// so that the buffer a step reads is always the one that holds its state
hipError_t launch_batch_tick(int64_t* t_dev, CaseRec* cases, int n_cases, const int* active, hipStream_t st);
hipError_t launch_batch_set_time(int64_t* t_dev, int64_t t, CaseRec* cases, int n_cases, hipStream_t st);
// A sampling step: clear every case's partials (max_parts: the most any case
// has), step with sample set, then sum each active case's partials per row
// and reduce them to the record at n_rec[case] of its ring; a record that
// fails the guard switches its case off.
hipError_t launch_batch_sample_begin(const CaseRec* cases, int n_cases, size_t max_parts, hipStream_t st);
hipError_t launch_batch_sample_end(const CaseRec* cases, int n_cases, int max_ny, const int64_t* t_dev, int64_t* n_rec,
                                   int* active, hipStream_t st);
// workgroups of the plain batched kernel that are resident at once on the
// current device (0 on error)
int batch_resident_workgroups(int waves_x);

} // namespace ij
