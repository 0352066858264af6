// ij_api.cpp -- host side of the C ABI declared in include/inkjet_lbm.h:
// parameter validation, derivation of the model constants (double precision,
// rounded once to float), device memory, the step loop with the pulse
// schedule, and the droplet-diagnostics summary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ij_internal.h"

using ij::KParams;
using namespace ij_host;

namespace {
thread_local std::string g_create_error;
}  // namespace

namespace ij_host {

ij_status fail(ij_sim* s, ij_status st, const std::string& msg)
{
    if (s)
        s->err = msg;
    else
        g_create_error = msg;
    return st;
}

ij_status hip_fail(ij_sim* s, hipError_t e, const char* where)
{
    return fail(s, IJ_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define IJ_HIP(s, call)                                 \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(s, e_, #call); \
    } while (0)

// Wetting parameter Omega from the contact angle (degrees, through the ink):
// inverse of cos(theta) = [(1+Omega)^{3/2} - (1-Omega)^{3/2}]/2, the Cahn
// wetting relation of the phi^4 free energy.  Closed form via the cubic in
// cos(alpha/3) with alpha = arccos(sin^2 theta).
double wetting_omega(double theta_deg)
{
    if (theta_deg == 90.0) return 0.0;
    const double th = theta_deg * M_PI / 180.0;
    const double s2 = std::sin(th) * std::sin(th);
    const double c = std::cos(std::acos(std::min(1.0, s2)) / 3.0);
    const double mag = 2.0 * std::sqrt(std::max(0.0, c * (1.0 - c)));
    return theta_deg < 90.0 ? mag : -mag;
}

// Fig. 1 pulse: +f_pos on [0, t_pos), -f_neg on [t_pos, t_pos + t_neg), then
// idle; periodic with period t_pos + t_neg + t_idle when requested.
double pulse_value(const ij_params& p, int64_t t)
{
    const int64_t period = p.t_pos + p.t_neg + p.t_idle;
    int64_t tt = t;
    if (p.periodic_pulse && period > 0) tt = t % period;
    if (tt < p.t_pos) return p.f_pos;
    if (tt < p.t_pos + p.t_neg) return -p.f_neg;
    return 0.0;
}

std::string validate(const ij_params& p)
{
    if (p.nx < 3 || p.ny < 3) return "nx and ny must be >= 3";
    if (p.nx > (1 << 24) || p.ny > 65535) return "lattice dimension too large (ny <= 65535)";
    if (p.bc_y != IJ_BC_PERIODIC && p.bc_y != IJ_BC_OPEN) return "bc_y must be IJ_BC_PERIODIC or IJ_BC_OPEN";
    if (!(p.tau_ink > 0.5) || !(p.tau_amb > 0.5) || !(p.tau_phi > 0.5)) return "relaxation times must exceed 1/2";
    if (!(p.rho_amb > 0.0) || !(p.rho_ink > p.rho_amb)) return "need rho_ink > rho_amb > 0";
    if (!(p.width > 0.0)) return "interface width must be positive";
    if (!(p.sigma >= 0.0)) return "surface tension must be >= 0";
    if (!(p.gamma >= 0.0)) return "mobility Gamma must be >= 0";
    if (!(p.theta_inner >= 0.0 && p.theta_inner <= 180.0) || !(p.theta_outer >= 0.0 && p.theta_outer <= 180.0))
        return "contact angles must lie in [0, 180]";
    if (p.t_pos < 0 || p.t_neg < 0 || p.t_idle < 0) return "pulse durations must be >= 0";
    if (!std::isfinite(p.f_pos) || !std::isfinite(p.f_neg)) return "pulse amplitudes must be finite";
    if (p.nozzle_w < 0 || (p.nozzle_w > 0 && (p.nozzle_x0 < 1 || p.nozzle_x0 + p.nozzle_w > p.nx - 1 ||
                                               p.nozzle_len < 1 || p.nozzle_len > p.ny - 2)))
        return "nozzle must lie inside the lattice with a wall column on each side";
    if (p.diag_row0 < 0 || p.diag_row0 >= p.ny) return "diag_row0 outside the lattice";
    if (p.diag_every < 0) return "diag_every must be >= 0";
    const double planes = 15.0 * (double)p.ny * (double)round_up(p.nx, kPitchAlign);
    if (planes >= 2147483647.0) return "lattice too large for 32-bit plane offsets";
    return "";
}

std::string check_wall(const ij_params& p, const uint8_t* w)
{
    const int64_t nx = p.nx, ny = p.ny;
    for (int64_t k = 0; k < nx * ny; ++k)
        if (w[k] > 2) return "wall mask values must be 0, 1 or 2";
    if (p.bc_y == IJ_BC_OPEN)
        for (int64_t x = 0; x < nx; ++x) {
            if (w[x] == 0 && w[nx + x] != 0) return "open bottom row: fluid node without fluid above";
            if (w[(ny - 1) * nx + x] == 0 && w[(ny - 2) * nx + x] != 0)
                return "open top row: fluid node without fluid below";
        }
    return "";
}

void build_nozzle(const ij_params& p, std::vector<uint8_t>& w)
{
    const int64_t nx = p.nx, ny = p.ny;
    w.assign((size_t)(nx * ny), IJ_FLUID);
    if (p.nozzle_w <= 0) return;
    for (int64_t y = 0; y < p.nozzle_len; ++y)
        for (int64_t x = 0; x < nx; ++x) {
            uint8_t v = IJ_WALL_OUTER;
            if (x >= p.nozzle_x0 && x < p.nozzle_x0 + p.nozzle_w) v = IJ_FLUID;
            if (x == p.nozzle_x0 - 1 || x == p.nozzle_x0 + p.nozzle_w) v = IJ_WALL_INNER;
            w[(size_t)(y * nx + x)] = v;
        }
}

void fill_kparams(ij_sim* s)
{
    KParams& K = s->K;
    const ij_params& p = s->p;
    K.nx = s->nx;
    K.ny = s->ny;
    K.pitch = s->pitch;
    K.bc_open = p.bc_y == IJ_BC_OPEN;
    K.force_rows = (int)std::min<int64_t>(p.force_rows, s->ny);
    K.diag_row0 = (int)p.diag_row0;
    K.plane = (unsigned)s->plane;
    K.rs = (unsigned)(ij::kFloatPlanes * s->pitch + s->pitch / 2);   // 14 float rows and one 16-bit row
    K.phi_star = s->phi_star;
    K.beta4 = 4.0 * s->beta;
    K.kappa = s->kappa;
    K.gamma = p.gamma;
    K.omega_phi = 1.0 / p.tau_phi;
    K.inv_width = 1.0 / p.width;
    K.wet[0] = 0.0;
    K.wet[1] = s->wet_in;
    K.wet[2] = s->wet_out;
    K.wet[3] = 0.0;
    K.n0 = (float)s->n0;
    K.inv_phi_star = (float)(1.0 / s->phi_star);
    K.tau_amb = (float)p.tau_amb;
    K.dtau = (float)(p.tau_ink - p.tau_amb);
    K.omq = (float)(1.0 - s->q);
    K.c_half_q = (float)(1.0 / (2.0 * s->q));
    K.omega_phi_f = (float)(1.0 / p.tau_phi);
    K.gamma_f = (float)p.gamma;
    K.fb = 0.f;
}

ij_status build_plain(ij_sim* s);

ij_status upload_wall(ij_sim* s)
{
    // padded device copy and the list of solid nodes with a fluid neighbour
    std::vector<uint8_t> padded((size_t)s->ny * s->pitch, IJ_WALL_OUTER);
    for (int y = 0; y < s->ny; ++y)
        std::memcpy(&padded[(size_t)y * s->pitch], &s->wall_host[(size_t)y * s->nx], (size_t)s->nx);
    IJ_HIP(s, hipMemcpy(s->wall, padded.data(), padded.size(), hipMemcpyHostToDevice));
    std::vector<int2> list;
    const bool open = s->p.bc_y == IJ_BC_OPEN;
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            if (s->wall_host[(size_t)y * s->nx + x] == 0) continue;
            bool touches = false;
            for (int dy = -1; dy <= 1 && !touches; ++dy)
                for (int dx = -1; dx <= 1 && !touches; ++dx) {
                    int yy = y + dy;
                    if (yy < 0 || yy >= s->ny) {
                        if (open) continue;
                        yy = (yy + s->ny) % s->ny;
                    }
                    const int xx = (x + dx + s->nx) % s->nx;
                    if (s->wall_host[(size_t)yy * s->nx + xx] == 0) touches = true;
                }
            if (touches) list.push_back(make_int2(x, y));
        }
    if (s->ghost) {
        (void)hipFree(s->ghost);
        s->ghost = nullptr;
    }
    s->n_ghost = (int)list.size();
    if (s->n_ghost) {
        if (hipMalloc(&s->ghost, list.size() * sizeof(int2)) != hipSuccess)
            return fail(s, IJ_ERR_OOM, "ghost list allocation failed");
        IJ_HIP(s, hipMemcpy(s->ghost, list.data(), list.size() * sizeof(int2), hipMemcpyHostToDevice));
    }
    s->initialised = false;
    return build_plain(s);
}

// Plain rows: for strip k (columns [x0, x0 + w) with two halo columns each
// side; strips are 64 * waves_x columns wide, and with mixed strips the
// columns past the last full one go to 64-column strips) row r is plain
// when rows r-1..r+1 hold no solid node in those columns and, with open
// rows, 1 <= r <= ny-2.  Tiles (strip, block of rows) that contain any
// other row go to the general launch.
ij_status build_plain(ij_sim* s)
{
    const int nx = s->nx, ny = s->ny;
    const int bw = 64 * s->waves_x;
    // strips of bw columns; with mixed strips the columns past the last full
    // one go to strips of 64 (one wave) instead of a partly idle wide strip
    const int n_wide = s->mixed_strips ? nx / bw : (nx + bw - 1) / bw;
    const int n_strips = n_wide + (s->mixed_strips ? (nx - n_wide * bw + 63) / 64 : 0);
    auto strip_x0 = [&](int k) { return k < n_wide ? k * bw : n_wide * bw + (k - n_wide) * 64; };
    auto strip_w = [&](int k) { return std::min(k < n_wide ? bw : 64, nx - strip_x0(k)); };
    const bool open = s->p.bc_y == IJ_BC_OPEN;
    // rows with any solid node in a column window: per strip
    std::vector<uint8_t> plain((size_t)n_strips * ny, 0);
    for (int k = 0; k < n_strips; ++k) {
        const int x0 = strip_x0(k), w = strip_w(k);
        std::vector<uint8_t> solid_row(ny, 0);
        for (int y = 0; y < ny; ++y)
            for (int c = x0 - 2; c < x0 + w + 2 && !solid_row[y]; ++c)
                if (s->wall_host[(size_t)y * nx + ((c % nx) + nx) % nx] != 0) solid_row[y] = 1;
        for (int y = 0; y < ny; ++y) {
            bool ok = !(open && (y < 1 || y > ny - 2));
            for (int dy = -1; dy <= 1 && ok; ++dy) {
                int r = y + dy;
                if (r < 0 || r >= ny) {
                    if (open) { ok = false; break; }
                    r = (r + ny) % ny;
                }
                if (solid_row[r]) ok = false;
            }
            plain[(size_t)k * ny + y] = ok ? 1 : 0;
        }
    }
    // general pieces, 64 columns wide (one wave): in each 64-column piece of
    // a strip, the runs of rows that are not plain and hold a fluid node in
    // the piece's columns, cut into pieces of at most kGeneralRows rows of
    // near-equal height.  A lone such row (an open row, the row above a
    // nozzle plate) is one piece of one row.  Pieces are short (latency: a
    // lone lattice leaves the device mostly idle) unless the lattice is one
    // of a batch (throughput) and some strip has a long run of general rows.
    int longest = 0;
    for (int k = 0; k < n_strips; ++k)
        for (int y = 0, run = 0; y < ny; ++y) {
            run = plain[(size_t)k * ny + y] ? 0 : run + 1;
            longest = std::max(longest, run);
        }
    const int kGeneralRows = s->in_batch && longest >= kGeneralTallRun ? kGeneralRowsTall : kGeneralRowsShort;
    std::vector<int4> gt;   // (strip, first row, first column, rows)
    std::vector<uint8_t> take((size_t)ny);
    for (int k = 0; k < n_strips; ++k) {
        const int sx0 = strip_x0(k), sx1 = sx0 + strip_w(k);
        for (int c0 = sx0; c0 < sx1; c0 += 64) {
            const int c1 = std::min(sx1, c0 + 64);
            for (int y = 0; y < ny; ++y) {
                bool fluid = false;
                if (!plain[(size_t)k * ny + y])
                    for (int x = c0; x < c1 && !fluid; ++x) fluid = s->wall_host[(size_t)y * nx + x] == 0;
                take[(size_t)y] = fluid ? 1 : 0;
            }
            for (int r0 = 0; r0 < ny;) {
                if (!take[(size_t)r0]) {
                    ++r0;
                    continue;
                }
                int r1 = r0;
                while (r1 < ny && take[(size_t)r1]) ++r1;
                const int n = r1 - r0, parts = (n + kGeneralRows - 1) / kGeneralRows;
                for (int j = 0, y0 = r0; j < parts; ++j) {
                    const int h = n / parts + (j < n % parts ? 1 : 0);
                    gt.push_back(make_int4(k, y0, c0, h));
                    y0 += h;
                }
                r0 = r1;
            }
        }
    }
    // row-major order: pieces that share halo rows run close together
    std::stable_sort(gt.begin(), gt.end(), [](const int4& a, const int4& b) {
        return a.y != b.y ? a.y < b.y : (a.x != b.x ? a.x < b.x : a.z < b.z);
    });
    s->n_strips = n_strips;
    s->n_wide = n_wide;
    s->n_rb = (ny + s->rows_per_block - 1) / s->rows_per_block;
    // plain tiles that hold a plain row; when some do not (a block of rows
    // that all sit beside solid nodes, such as a nozzle channel), the plain
    // launch runs over the list of the others
    s->tile_plain.assign((size_t)s->n_rb * n_strips, 0);
    std::vector<int4> pt;   // (strip, first row, first column, rows)
    for (int b = 0; b < s->n_rb; ++b)
        for (int k = 0; k < n_strips; ++k) {
            const int y0 = b * s->rows_per_block, y1 = std::min(ny, y0 + s->rows_per_block);
            bool any = false;
            for (int y = y0; y < y1 && !any; ++y) any = plain[(size_t)k * ny + y] != 0;
            s->tile_plain[(size_t)b * n_strips + k] = any ? 1 : 0;
            if (any) pt.push_back(make_int4(k, y0, strip_x0(k), y1 - y0));
        }
    if (s->ptiles) (void)hipFree(s->ptiles);
    s->ptiles = nullptr;
    s->n_ptiles = -1;
    if (!s->in_batch && !s->mixed_strips && pt.size() < s->tile_plain.size()) {
        if (!pt.empty()) {
            if (hipMalloc(&s->ptiles, pt.size() * sizeof(int4)) != hipSuccess)
                return fail(s, IJ_ERR_OOM, "tile list allocation failed");
            IJ_HIP(s, hipMemcpy(s->ptiles, pt.data(), pt.size() * sizeof(int4), hipMemcpyHostToDevice));
        }
        s->n_ptiles = (int)pt.size();
    }
    s->strip_x0.resize((size_t)n_strips);
    for (int k = 0; k < n_strips; ++k) s->strip_x0[(size_t)k] = strip_x0(k);
    s->gtiles_host = gt;
    s->plain_host = plain;
    if (s->plain) (void)hipFree(s->plain);
    if (s->gtiles) (void)hipFree(s->gtiles);
    s->plain = nullptr;
    s->gtiles = nullptr;
    if (hipMalloc(&s->plain, plain.size()) != hipSuccess) return fail(s, IJ_ERR_OOM, "plain-row table allocation failed");
    IJ_HIP(s, hipMemcpy(s->plain, plain.data(), plain.size(), hipMemcpyHostToDevice));
    s->n_gtiles = (int)gt.size();
    if (s->n_gtiles) {
        if (hipMalloc(&s->gtiles, gt.size() * sizeof(int4)) != hipSuccess)
            return fail(s, IJ_ERR_OOM, "tile list allocation failed");
        IJ_HIP(s, hipMemcpy(s->gtiles, gt.data(), gt.size() * sizeof(int4), hipMemcpyHostToDevice));
    }
    return IJ_OK;
}

// stability guard of the diagnostics samples: non-finite nodes or max |u|
// above this limit
double u_limit(const ij_params& p) { return p.u_limit > 0 ? p.u_limit : 0.3; }

int diag_band(double width) { return std::max(1, (int)std::ceil(width - 1e-9)); }

ij_status drain_samples(ij_sim* s, hipStream_t st)
{
    if (s->n_dev_samples == 0) return IJ_OK;
    std::vector<ij::SampleRec> tmp((size_t)s->n_dev_samples);
    IJ_HIP(s, hipMemcpyAsync(tmp.data(), s->samples, tmp.size() * sizeof(ij::SampleRec), hipMemcpyDeviceToHost, st));
    IJ_HIP(s, hipStreamSynchronize(st));
    static_assert(sizeof(ij::SampleRec) == sizeof(ij_sample), "sample layouts differ");
    for (const auto& r : tmp) {
        ij_sample o;
        std::memcpy(&o, &r, sizeof o);
        s->host_samples.push_back(o);
        if (s->unstable_step < 0 && (o.nan_count > 0 || !(o.max_u <= u_limit(s->p)))) {
            s->unstable_step = o.step;
            // A batch switches such a case off on the device at the same
            // sample: its state stays in the buffer that was current at that
            // step, while the host went on alternating its buffers.
            if (s->in_batch) s->cur ^= (int)((s->t - o.step) & 1);
        }
    }
    s->n_dev_samples = 0;
    return IJ_OK;
}

ij_status record_sample(ij_sim* s, hipStream_t st)
{
    if (s->n_dev_samples >= kSampleCap) {
        ij_status r = drain_samples(s, st);
        if (r != IJ_OK) return r;
    }
    s->K.fb = (float)pulse_value(s->p, s->t);
    hipError_t e = ij::launch_phi_ghost(s->K, s->buf[s->cur], s->wall, s->phi, s->ghost, s->n_ghost, st);
    if (e != hipSuccess) return hip_fail(s, e, "phi/ghost kernels");
    const int a_min = (int)std::ceil(4.0 * s->p.width * s->p.width);
    e = ij::launch_diag(s->K, s->buf[s->cur], s->wall, s->phi, (int)s->p.diag_row0, a_min, diag_band(s->p.width),
                        s->t, s->rows, s->samples + s->n_dev_samples, st);
    if (e != hipSuccess) return hip_fail(s, e, "diagnostics kernels");
    s->n_dev_samples += 1;
    return IJ_OK;
}

}  // namespace ij_host

void ij_host::destroy_sim(ij_sim* s)
{
    if (!s) return;
    for (int b = 0; b < 2; ++b)
        if (s->own[b] && s->buf[b]) (void)hipFree(s->buf[b]);
    if (s->wall) (void)hipFree(s->wall);
    if (s->phi) (void)hipFree(s->phi);
    if (s->ghost) (void)hipFree(s->ghost);
    if (s->rows) (void)hipFree(s->rows);
    if (s->samples) (void)hipFree(s->samples);
    if (s->plain) (void)hipFree(s->plain);
    if (s->gtiles) (void)hipFree(s->gtiles);
    if (s->ptiles) (void)hipFree(s->ptiles);
    if (s->sample_parts) (void)hipFree(s->sample_parts);
    delete s;
}

extern "C" {

ij_status ij_params_default(ij_params* p)
{
    if (!p) return IJ_ERR_INVALID_ARG;
    std::memset(p, 0, sizeof *p);
    p->nx = 64;
    p->ny = 256;
    p->bc_y = IJ_BC_OPEN;
    p->nozzle_x0 = 24;
    p->nozzle_w = 16;
    p->nozzle_len = 64;
    p->force_rows = 64;
    p->diag_row0 = 64;
    p->rho_ink = 1.0;
    p->rho_amb = 0.1;
    p->sigma = 0.01;
    p->width = 4.0;
    p->gamma = 1.0;
    p->tau_ink = p->tau_amb = p->tau_phi = 1.0;
    p->theta_inner = p->theta_outer = 90.0;
    p->u_limit = 0.3;
    return IJ_OK;
}

ij_status ij_required_bytes(const ij_params* p, size_t* bytes)
{
    if (!p || !bytes) return IJ_ERR_INVALID_ARG;
    const std::string v = validate(*p);
    if (!v.empty()) return fail(nullptr, IJ_ERR_INVALID_ARG, v);
    *bytes = buffer_bytes((size_t)p->ny * (size_t)round_up(p->nx, kPitchAlign));
    return IJ_OK;
}

ij_status ij_create(const ij_params* p, ij_sim** out)
{
    if (!out) return fail(nullptr, IJ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!p) return fail(nullptr, IJ_ERR_INVALID_ARG, "params is NULL");
    const std::string v = validate(*p);
    if (!v.empty()) return fail(nullptr, IJ_ERR_INVALID_ARG, v);

    ij_sim* s = new ij_sim();
    s->p = *p;
    s->nx = (int)p->nx;
    s->ny = (int)p->ny;
    s->pitch = (int)round_up(p->nx, kPitchAlign);
    s->plane = (size_t)s->ny * s->pitch;
    // composition variables (Eqs. 1, 7): n = (rho_A + rho_B)/2, phi = (rho_A - rho_B)/2
    s->phi_star = 0.5 * (p->rho_ink - p->rho_amb);
    s->n0 = 0.5 * (p->rho_ink + p->rho_amb);
    // phi^4 closure: profile phi* tanh(2z/W) with tension sigma
    const double ps2 = s->phi_star * s->phi_star;
    s->beta = 3.0 * p->sigma / (4.0 * p->width * ps2 * ps2);
    s->kappa = 3.0 * p->sigma * p->width / (8.0 * ps2);
    s->q = 1.0 / (p->tau_phi + 0.5);
    s->wet_in = 2.0 * wetting_omega(p->theta_inner) * s->phi_star / p->width;
    s->wet_out = 2.0 * wetting_omega(p->theta_outer) * s->phi_star / p->width;
    if (s->p.force_rows == 0 && p->nozzle_w > 0) s->p.force_rows = p->nozzle_len;
    fill_kparams(s);

    const size_t bytes = buffer_bytes(s->plane);
    auto cleanup = [&](ij_status st, const std::string& m) {
        const std::string msg = m;
        ij_destroy(s);
        return fail(nullptr, st, msg);
    };
    for (int b = 0; b < 2; ++b) {
        if (hipMalloc(&s->buf[b], bytes) != hipSuccess) return cleanup(IJ_ERR_OOM, "distribution buffer allocation failed");
        s->own[b] = true;
    }
    if (hipMalloc(&s->wall, s->plane) != hipSuccess || hipMalloc(&s->phi, s->plane * sizeof(double)) != hipSuccess ||
        hipMalloc(&s->rows, (size_t)s->ny * sizeof(ij::DiagRow)) != hipSuccess ||
        hipMalloc(&s->samples, (size_t)kSampleCap * sizeof(ij::SampleRec)) != hipSuccess)
        return cleanup(IJ_ERR_OOM, "scratch allocation failed");
    if (hipMemset(s->phi, 0, s->plane * sizeof(double)) != hipSuccess)
        return cleanup(IJ_ERR_DEVICE, "hipMemset failed");
    build_nozzle(s->p, s->wall_host);
    const std::string wv = check_wall(s->p, s->wall_host.data());
    if (!wv.empty()) return cleanup(IJ_ERR_INVALID_ARG, wv);
    if (upload_wall(s) != IJ_OK) return cleanup(IJ_ERR_DEVICE, s->err);
    *out = s;
    return IJ_OK;
}

void ij_destroy(ij_sim* s)
{
    if (!s || s->in_batch) return;   // batch members go with their batch
    ij_host::destroy_sim(s);
}


const char* ij_last_error(const ij_sim* s) { return s ? s->err.c_str() : g_create_error.c_str(); }

ij_status ij_attach_buffers(ij_sim* s, void* a, void* b, size_t bytes_each)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (s->in_batch) return fail(s, IJ_ERR_STATE, "a batch member keeps the buffers of its batch");
    if (!a || !b || a == b) return fail(s, IJ_ERR_INVALID_ARG, "need two distinct device buffers");
    const size_t need = buffer_bytes(s->plane);
    if (bytes_each < need) return fail(s, IJ_ERR_INVALID_ARG, "buffers smaller than ij_required_bytes");
    if (((uintptr_t)a & 255) || ((uintptr_t)b & 255)) return fail(s, IJ_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    for (int k = 0; k < 2; ++k)
        if (s->own[k] && s->buf[k]) {
            (void)hipFree(s->buf[k]);
            s->own[k] = false;
        }
    s->buf[0] = (float*)a;
    s->buf[1] = (float*)b;
    s->cur = 0;
    s->initialised = false;
    return IJ_OK;
}

ij_status ij_set_wall(ij_sim* s, const uint8_t* w)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (!w) return fail(s, IJ_ERR_INVALID_ARG, "wall is NULL");
    const std::string v = check_wall(s->p, w);
    if (!v.empty()) return fail(s, IJ_ERR_INVALID_ARG, v);
    s->wall_host.assign(w, w + (size_t)s->nx * s->ny);
    return upload_wall(s);
}

ij_status ij_set_solid_mask(ij_sim* s, const uint8_t* mask, int32_t on_device)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (!mask) return fail(s, IJ_ERR_INVALID_ARG, "mask is NULL");
    if (!on_device) return ij_set_wall(s, mask);
    // the host analysis (wall classes, ghost and tile lists) reads a host copy
    std::vector<uint8_t> h((size_t)s->nx * s->ny);
    const hipError_t e = hipMemcpy(h.data(), mask, h.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(s, e, "copy of the device mask");
    return ij_set_wall(s, h.data());
}

static ij_status do_init(ij_sim* s, const float* src, int from_distance, const float* ux, const float* uy,
                         void* stream)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (!src) return fail(s, IJ_ERR_INVALID_ARG, "initial field is NULL");
    hipStream_t st = (hipStream_t)stream;
    s->cur = 0;
    s->t = 0;
    s->K.fb = 0.f;
    hipError_t e = ij::launch_init(s->K, s->buf[0], s->wall, s->phi, src, from_distance, ux, uy, s->ghost,
                                   s->n_ghost, st);
    if (e != hipSuccess) return hip_fail(s, e, "init kernels");
    s->host_samples.clear();
    s->n_dev_samples = 0;
    s->unstable_step = -1;
    s->initialised = true;
    return IJ_OK;
}

ij_status ij_init_distance(ij_sim* s, const float* d, void* stream) { return do_init(s, d, 1, nullptr, nullptr, stream); }

ij_status ij_init_phi(ij_sim* s, const float* phi, const float* ux, const float* uy, void* stream)
{
    return do_init(s, phi, 0, ux, uy, stream);
}

ij_status ij_init_default(ij_sim* s, void* stream)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    const int64_t L = s->p.nozzle_w > 0 ? s->p.nozzle_len : s->ny / 4;
    std::vector<float> d((size_t)s->nx * s->ny);
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) d[(size_t)y * s->nx + x] = (float)((double)L - 0.5 - y);
    float* dd = nullptr;
    IJ_HIP(s, hipMalloc(&dd, d.size() * sizeof(float)));
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(dd, d.data(), d.size() * sizeof(float), hipMemcpyHostToDevice, st);
    ij_status r = e == hipSuccess ? do_init(s, dd, 1, nullptr, nullptr, stream) : hip_fail(s, e, "hipMemcpyAsync");
    (void)hipStreamSynchronize(st);
    (void)hipFree(dd);
    return r;
}

ij_status ij_step(ij_sim* s, int64_t nsteps, void* stream)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (s->in_batch) return fail(s, IJ_ERR_STATE, "a batch member is stepped by its batch (ij_batch_step)");
    if (!s->initialised) return fail(s, IJ_ERR_STATE, "step before init");
    if (nsteps < 0) return fail(s, IJ_ERR_INVALID_ARG, "nsteps < 0");
    if (s->unstable_step >= 0) return fail(s, IJ_ERR_UNSTABLE, "a diagnostics sample failed the stability guard");
    hipStream_t st = (hipStream_t)stream;
    const int n_sub = (s->nx + 63) / 64;
    const size_t n_parts = (size_t)n_sub * (size_t)s->ny;
    for (int64_t k = 0; k < nsteps; ++k) {
        // a step at a sampling time also takes the sample of its input state
        // (the collide kernels emit per-piece row partials), instead of a
        // separate pass over the lattice
        const bool sample = s->p.diag_every > 0 && s->t % s->p.diag_every == 0;
        if (sample) {
            if (s->n_dev_samples >= kSampleCap) {
                ij_status r = drain_samples(s, st);
                if (r != IJ_OK) return r;
            }
            if (!s->sample_parts && hipMalloc(&s->sample_parts, n_parts * sizeof(ij::DiagRow)) != hipSuccess) {
                s->sample_parts = nullptr;
                return fail(s, IJ_ERR_OOM, "sample partials allocation failed");
            }
            const hipError_t e = ij::launch_sample_clear(s->sample_parts, n_parts, st);
            if (e != hipSuccess) return hip_fail(s, e, "sample clear kernel");
        }
        s->K.fb = (float)pulse_value(s->p, s->t);
        hipError_t e = ij::launch_collide_fused(s->K, s->buf[s->cur], s->buf[1 - s->cur], s->wall, s->plain,
                                                s->ptiles, s->n_ptiles, s->gtiles, s->n_gtiles, s->waves_x,
                                                s->rows_per_block, sample ? s->sample_parts : nullptr, st);
        if (e != hipSuccess) return hip_fail(s, e, "collide-stream kernel");
        if (sample) {
            const int a_min = (int)std::ceil(4.0 * s->p.width * s->p.width);
            e = ij::launch_sample_finish(s->sample_parts, n_sub, s->ny, (int)s->p.diag_row0, a_min,
                                         diag_band(s->p.width), s->t, s->rows, s->samples + s->n_dev_samples, st);
            if (e != hipSuccess) return hip_fail(s, e, "diagnostics kernels");
            s->n_dev_samples += 1;
        }
        s->cur = 1 - s->cur;
        s->t += 1;
    }
    return IJ_OK;
}

// Reference path (one node per thread, phi round trip through memory); kept
// for cross-checking the fused kernel.
ij_status ij_step_reference(ij_sim* s, int64_t nsteps, void* stream)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (s->in_batch) return fail(s, IJ_ERR_STATE, "a batch member is stepped by its batch (ij_batch_step)");
    if (!s->initialised) return fail(s, IJ_ERR_STATE, "step before init");
    hipStream_t st = (hipStream_t)stream;
    for (int64_t k = 0; k < nsteps; ++k) {
        s->K.fb = (float)pulse_value(s->p, s->t);
        hipError_t e = ij::launch_phi_ghost(s->K, s->buf[s->cur], s->wall, s->phi, s->ghost, s->n_ghost, st);
        if (e == hipSuccess)
            e = ij::launch_collide_ref(s->K, s->buf[s->cur], s->buf[1 - s->cur], s->wall, s->phi, st);
        if (e != hipSuccess) return hip_fail(s, e, "reference kernels");
        s->cur = 1 - s->cur;
        s->t += 1;
    }
    return IJ_OK;
}

int64_t ij_time(const ij_sim* s) { return s ? s->t : -1; }

ij_status ij_get_moments(ij_sim* s, float* n, float* ph, float* ux, float* uy, void* stream)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (!s->initialised) return fail(s, IJ_ERR_STATE, "moments before init");
    hipStream_t st = (hipStream_t)stream;
    if (s->in_batch) {   // the buffer of a case the batch froze is known once its samples are read
        const ij_status r = drain_samples(s, st);
        if (r != IJ_OK) return r;
    }
    s->K.fb = (float)pulse_value(s->p, s->t);
    hipError_t e = ij::launch_phi_ghost(s->K, s->buf[s->cur], s->wall, s->phi, s->ghost, s->n_ghost, st);
    if (e == hipSuccess) e = ij::launch_moments(s->K, s->buf[s->cur], s->wall, s->phi, n, ph, ux, uy, st);
    if (e != hipSuccess) return hip_fail(s, e, "moment kernels");
    return IJ_OK;
}

ij_status ij_get_state(ij_sim* s, float* f, float* g, void* stream)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (!s->initialised) return fail(s, IJ_ERR_STATE, "state before init");
    if (s->in_batch) {   // the buffer of a case the batch froze is known once its samples are read
        const ij_status r = drain_samples(s, (hipStream_t)stream);
        if (r != IJ_OK) return r;
    }
    hipError_t e = ij::launch_state_io(s->K, s->buf[s->cur], s->wall, f, g, 1, (hipStream_t)stream);
    return e == hipSuccess ? IJ_OK : hip_fail(s, e, "state readback kernel");
}

ij_status ij_set_state(ij_sim* s, const float* f, const float* g, int64_t t, void* stream)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (!f || !g) return fail(s, IJ_ERR_INVALID_ARG, "f and g are required");
    if (t < 0) return fail(s, IJ_ERR_INVALID_ARG, "t < 0");
    hipError_t e = ij::launch_state_io(s->K, s->buf[s->cur], s->wall, (float*)f, (float*)g, 0, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(s, e, "state write kernel");
    s->t = t;
    s->initialised = true;
    return IJ_OK;
}

ij_status ij_state_bytes(const ij_sim* s, size_t* bytes)
{
    if (!s || !bytes) return IJ_ERR_INVALID_ARG;
    *bytes = sizeof(StateHeader) + buffer_bytes(s->plane);
    return IJ_OK;
}

ij_status ij_save_state(ij_sim* s, void* blob, size_t bytes, void* stream)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (!blob) return fail(s, IJ_ERR_INVALID_ARG, "blob is NULL");
    if (!s->initialised) return fail(s, IJ_ERR_STATE, "state before init");
    const size_t payload = buffer_bytes(s->plane);
    if (bytes < sizeof(StateHeader) + payload) return fail(s, IJ_ERR_INVALID_ARG, "blob smaller than ij_state_bytes");
    hipStream_t st = (hipStream_t)stream;
    if (s->in_batch) {   // the buffer of a case the batch froze is known once its samples are read
        const ij_status r = drain_samples(s, st);
        if (r != IJ_OK) return r;
    }
    StateHeader h{};
    std::memcpy(h.magic, "IJSTATE3", 8);
    h.nx = s->nx;
    h.ny = s->ny;
    h.nz = 1;
    h.pitch = s->pitch;
    h.t = s->t;
    h.wall_hash = fnv1a(s->wall_host.data(), s->wall_host.size());
    h.payload = payload;
    std::memcpy(blob, &h, sizeof h);
    IJ_HIP(s, hipMemcpyAsync((char*)blob + sizeof h, s->buf[s->cur], payload, hipMemcpyDeviceToHost, st));
    IJ_HIP(s, hipStreamSynchronize(st));
    return IJ_OK;
}

ij_status ij_load_state(ij_sim* s, const void* blob, size_t bytes, void* stream)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (!blob || bytes < sizeof(StateHeader)) return fail(s, IJ_ERR_INVALID_ARG, "blob is NULL or too small");
    StateHeader h;
    std::memcpy(&h, blob, sizeof h);
    const size_t payload = buffer_bytes(s->plane);
    if (std::memcmp(h.magic, "IJSTATE3", 8) != 0) return fail(s, IJ_ERR_INVALID_ARG, "not a checkpoint of this library");
    if (h.nx != s->nx || h.ny != s->ny || h.nz != 1 || h.pitch != s->pitch || h.payload != payload)
        return fail(s, IJ_ERR_INVALID_ARG, "checkpoint of a different lattice size");
    if (h.wall_hash != fnv1a(s->wall_host.data(), s->wall_host.size()))
        return fail(s, IJ_ERR_INVALID_ARG, "checkpoint of a different wall mask");
    if (h.t < 0) return fail(s, IJ_ERR_INVALID_ARG, "negative step counter");
    if (bytes < sizeof h + payload) return fail(s, IJ_ERR_INVALID_ARG, "blob shorter than its payload");
    hipStream_t st = (hipStream_t)stream;
    IJ_HIP(s, hipMemcpyAsync(s->buf[0], (const char*)blob + sizeof h, payload, hipMemcpyHostToDevice, st));
    IJ_HIP(s, hipStreamSynchronize(st));
    s->cur = 0;
    s->t = h.t;
    s->initialised = true;
    s->host_samples.clear();
    s->n_dev_samples = 0;
    s->unstable_step = -1;
    return IJ_OK;
}

ij_status ij_diag_sample(ij_sim* s, void* stream)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (!s->initialised) return fail(s, IJ_ERR_STATE, "diagnostics before init");
    if (s->in_batch) {
        const ij_status r = drain_samples(s, (hipStream_t)stream);
        if (r != IJ_OK) return r;
    }
    return record_sample(s, (hipStream_t)stream);
}

ij_status ij_get_row_profile(ij_sim* s, int64_t* count, double* uy, void* stream)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (s->n_dev_samples == 0 && s->host_samples.empty()) return fail(s, IJ_ERR_STATE, "no diagnostics sample yet");
    hipStream_t st = (hipStream_t)stream;
    std::vector<ij::DiagRow> rows((size_t)s->ny);
    IJ_HIP(s, hipMemcpyAsync(rows.data(), s->rows, rows.size() * sizeof(ij::DiagRow), hipMemcpyDeviceToHost, st));
    IJ_HIP(s, hipStreamSynchronize(st));
    for (int y = 0; y < s->ny; ++y) {
        if (count) count[y] = rows[(size_t)y].count;
        if (uy) uy[y] = rows[(size_t)y].uy;
    }
    return IJ_OK;
}

ij_status ij_get_samples(ij_sim* s, ij_sample* out, int64_t cap, int64_t* count, void* stream)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    ij_status r = drain_samples(s, (hipStream_t)stream);
    if (r != IJ_OK) return r;
    const int64_t n = (int64_t)s->host_samples.size();
    if (count) *count = n;
    if (out)
        for (int64_t k = 0; k < std::min(n, cap); ++k) out[k] = s->host_samples[(size_t)k];
    return IJ_OK;
}

ij_status ij_check(ij_sim* s, void* stream)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    ij_status r = drain_samples(s, (hipStream_t)stream);
    if (r != IJ_OK) return r;
    return s->unstable_step >= 0 ? fail(s, IJ_ERR_UNSTABLE, "a diagnostics sample failed the stability guard") : IJ_OK;
}

ij_status ij_get_diagnostics(ij_sim* s, ij_diag* out, void* stream)
{
    if (!s || !out) return IJ_ERR_INVALID_ARG;
    ij_status r = drain_samples(s, (hipStream_t)stream);
    if (r != IJ_OK) return r;
    std::memset(out, 0, sizeof *out);
    out->step = s->t;
    out->n_samples = (int64_t)s->host_samples.size();
    out->unstable_step = s->unstable_step;
    out->breakup_step = -1;
    out->v_drop = NAN;
    out->last.largest_top = -1;
    out->last.largest_bottom = -1;
    if (s->host_samples.empty()) return IJ_OK;
    out->last = s->host_samples.back();
    // breakup: first sample with a detached drop
    int64_t tb = -1;
    for (const auto& x : s->host_samples)
        if (x.n_detached > 0) {
            tb = x.step;
            out->drop_len = x.largest_top - x.largest_bottom + 1;   // drop and filament at breakup
            break;
        }
    out->breakup_step = tb;
    if (tb < 0) return IJ_OK;
    // drop velocity: mean of the largest drop's mean u_y over [tb+1000, tb+3000],
    // stopping once its top comes within 2W of the last row
    double acc = 0.0;
    int64_t nv = 0;
    for (const auto& x : s->host_samples) {
        if (x.step < tb + 1000 || x.step > tb + 3000 || x.largest_count <= 0) continue;
        if ((double)x.largest_top >= (double)(s->ny - 1) - 2.0 * s->p.width) break;
        acc += x.largest_uy / (double)x.largest_count;
        ++nv;
    }
    if (nv) out->v_drop = acc / (double)nv;
    for (const auto& x : s->host_samples)
        if (x.step >= tb + 2000) {
            out->vol_drop = x.largest_count;
            out->satellite = x.n_detached >= 2;
            break;
        }
    return IJ_OK;
}

ij_status ij_derived(const ij_sim* s, double out[8])
{
    if (!s || !out) return IJ_ERR_INVALID_ARG;
    out[0] = s->phi_star;
    out[1] = s->n0;
    out[2] = s->beta;
    out[3] = s->kappa;
    out[4] = s->q;
    out[5] = s->wet_in;
    out[6] = s->wet_out;
    out[7] = s->p.gamma * s->q * (s->q * s->p.tau_phi - 0.5);
    return IJ_OK;
}

ij_status ij_autotune(ij_sim* s, int32_t trial_steps, void* stream, int32_t* waves_x, int32_t* rows_per_block,
                      double* ms_per_step)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (s->in_batch) return fail(s, IJ_ERR_STATE, "a batch member takes the batch's tiling (ij_batch_autotune)");
    if (!s->initialised) return fail(s, IJ_ERR_STATE, "autotune before init");
    if (trial_steps < 2 || trial_steps > 10000) return fail(s, IJ_ERR_INVALID_ARG, "trial_steps must lie in [2, 10000]");
    hipStream_t st = (hipStream_t)stream;
    // rows_per_block 1: the row kernel (no walk) for plain rows
    static const int cand[][2] = {{1, 1},  {2, 1},  {4, 1},  {1, 8},  {1, 16}, {1, 32}, {2, 8},
                                  {2, 16}, {2, 32}, {4, 8},  {4, 16}, {4, 32}, {4, 64}};
    // trial steps run on the live buffers from a snapshot that is restored
    const size_t bytes = buffer_bytes(s->plane);
    void* saved = nullptr;
    if (hipMalloc(&saved, bytes) != hipSuccess) return fail(s, IJ_ERR_OOM, "autotune snapshot allocation failed");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMemcpyAsync(saved, s->buf[s->cur], bytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int old_w = s->waves_x, old_r = s->rows_per_block;
    int bw = old_w, br = old_r;
    double best = 1e300;
    trial_steps += trial_steps & 1;
    s->K.fb = (float)pulse_value(s->p, s->t);
    for (const auto& c : cand) {
        if (e != hipSuccess) break;
        s->waves_x = c[0];
        s->rows_per_block = c[1];
        if (build_plain(s) != IJ_OK) {
            e = hipErrorUnknown;
            break;
        }
        int cur = s->cur;
        auto steps = [&](int n) {
            hipError_t r = hipSuccess;
            for (int k = 0; k < n && r == hipSuccess; ++k) {
                r = ij::launch_collide_fused(s->K, s->buf[cur], s->buf[1 - cur], s->wall, s->plain, s->ptiles,
                                             s->n_ptiles, s->gtiles, s->n_gtiles, s->waves_x, s->rows_per_block,
                                             nullptr, st);
                cur = 1 - cur;
            }
            return r;
        };
        e = steps(2);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        if (e == hipSuccess) e = steps(trial_steps);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms / trial_steps < best) {
            best = ms / trial_steps;
            bw = c[0];
            br = c[1];
        }
    }
    (void)hipMemcpyAsync(s->buf[s->cur], saved, bytes, hipMemcpyDeviceToDevice, st);
    (void)hipStreamSynchronize(st);
    (void)hipFree(saved);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    s->waves_x = e == hipSuccess ? bw : old_w;
    s->rows_per_block = e == hipSuccess ? br : old_r;
    const ij_status r = build_plain(s);
    if (e != hipSuccess) return hip_fail(s, e, "autotune trial");
    if (r != IJ_OK) return r;
    if (waves_x) *waves_x = bw;
    if (rows_per_block) *rows_per_block = br;
    if (ms_per_step) *ms_per_step = best;
    return IJ_OK;
}

ij_status ij_set_tiling(ij_sim* s, int32_t waves_x, int32_t rows_per_block)
{
    if (!s) return IJ_ERR_INVALID_ARG;
    if (s->in_batch) return fail(s, IJ_ERR_STATE, "a batch member takes the batch's tiling (ij_batch_set_tiling)");
    if (waves_x != 0 && waves_x != 1 && waves_x != 2 && waves_x != 4)
        return fail(s, IJ_ERR_INVALID_ARG, "waves_x must be 1, 2 or 4");
    if (rows_per_block < 0 || rows_per_block > 1024)
        return fail(s, IJ_ERR_INVALID_ARG, "rows_per_block must lie in [0, 1024]");
    if (waves_x) s->waves_x = waves_x;
    if (rows_per_block) s->rows_per_block = rows_per_block;
    return build_plain(s);
}

}  // extern "C"
